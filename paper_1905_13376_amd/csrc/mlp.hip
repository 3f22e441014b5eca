// Learned planner: degree sketches of a join's relations and a small MLP
// (IN -> H -> H -> OUT, GELU) with BF16 weights and FP32 arithmetic, trained
// by the kernels below (forward, loss, backward, AdamW).
//
// Parameter buffer (device, caller-owned), MLP_PARAMS = P floats per block:
//   [ master fp32 P | grad fp32 P | adam m P | adam v P | bf16 weights ]
// with the parameters ordered W1 [H][IN], b1 [H], W2 [H][H], b2 [H],
// W3 [OUT][H], b3 [OUT].  The forward and backward passes read the BF16
// copies of W1, W2, W3 (biases stay FP32); AdamW updates the FP32 masters
// and refreshes the BF16 copies (round to nearest even).
//
// Sketch features (MLP_IN = 100): for R's B column, S's B column and T's C
// column, a 32-bin histogram of floor(log2 deg(v)) over the distinct keys v
// (bin value log2(1 + number of keys) / 32), then log2(1 + |R|), |S|, |T|
// (each / 32) and the kind (0 linear, 1 cyclic).
#include "mj_kernels.h"

namespace mj {

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float(uint32_t(h) << 16);
}
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    const uint32_t b = __float_as_uint(f);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float gelu_f(float x) {
    return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float x) {
    const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
    const float pdf = expf(-0.5f * x * x) * 0.39894228040143268f;
    return cdf + x * pdf;
}

// ------------------------------------------------------------------ forward
__global__ void __launch_bounds__(MLP_H)
k_mlp_fwd(MlpFwdArgs A) {
    __shared__ float x[MLP_IN], h1[MLP_H], h2[MLP_H];
    const uint32_t b = blockIdx.x, j = threadIdx.x;
    const float* P = A.params;
    const uint16_t* Wb = A.wbf16;
    for (uint32_t i = j; i < MLP_IN; i += MLP_H) x[i] = A.X[uint64_t(b) * MLP_IN + i];
    __syncthreads();
    float z1 = P[MLP_OFF_B1 + j];
    for (int i = 0; i < MLP_IN; ++i) z1 += bf16_to_f32(Wb[MLP_WB_W1 + j * MLP_IN + i]) * x[i];
    const float a1 = gelu_f(z1);
    h1[j] = a1;
    __syncthreads();
    float z2 = P[MLP_OFF_B2 + j];
    for (int k = 0; k < MLP_H; ++k) z2 += bf16_to_f32(Wb[MLP_WB_W2 + j * MLP_H + k]) * h1[k];
    const float a2 = gelu_f(z2);
    h2[j] = a2;
    if (A.act) {
        float* act = A.act + uint64_t(b) * MLP_ACT;
        act[j] = z1; act[MLP_H + j] = a1; act[2 * MLP_H + j] = z2; act[3 * MLP_H + j] = a2;
    }
    __syncthreads();
    if (j < MLP_OUT) {
        float y = P[MLP_OFF_B3 + j];
        for (int k = 0; k < MLP_H; ++k) y += bf16_to_f32(Wb[MLP_WB_W3 + j * MLP_H + k]) * h2[k];
        A.Y[uint64_t(b) * MLP_OUT + j] = y;
    }
}

// ------------------------------------------------------------------ loss
// one thread per sample: dY = dL/dY (already divided by B), loss += L_b / B
__global__ void k_mlp_loss(MlpLossArgs A) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= A.B) return;
    const float* y = A.Y + uint64_t(b) * MLP_OUT;
    float* g = A.dY + uint64_t(b) * MLP_OUT;
    const float invB = 1.0f / (float)A.B;
    float l = 0.f;
    for (int k = 0; k < 2; ++k) {
        const float d = y[k] - A.targets[2 * b + k];
        l += d * d;
        g[k] = 2.f * d * invB;
    }
    {   // plan head: softmax cross entropy over the MLP_NPLAN plan logits
        const float* z = y + MLP_PLAN0;
        float m = z[0];
        for (int k = 1; k < MLP_NPLAN; ++k) m = fmaxf(m, z[k]);
        float e[MLP_NPLAN], s = 0.f;
        for (int k = 0; k < MLP_NPLAN; ++k) { e[k] = expf(z[k] - m); s += e[k]; }
        const int c = A.plan_label[b];
        l += -(z[c] - m - logf(s));
        for (int k = 0; k < MLP_NPLAN; ++k) g[MLP_PLAN0 + k] = (e[k] / s - (k == c ? 1.f : 0.f)) * invB;
    }
    const int sc = A.share_label[b];
    if (sc >= 0) {
        const float* z = y + MLP_SHARE0;
        const float m = fmaxf(z[0], fmaxf(z[1], z[2]));
        const float e[3] = {expf(z[0] - m), expf(z[1] - m), expf(z[2] - m)};
        const float s = e[0] + e[1] + e[2];
        l += -(z[sc] - m - logf(s));
        for (int k = 0; k < 3; ++k) g[MLP_SHARE0 + k] = (e[k] / s - (k == sc ? 1.f : 0.f)) * invB;
    } else {
        g[MLP_SHARE0] = g[MLP_SHARE0 + 1] = g[MLP_SHARE0 + 2] = 0.f;
    }
    atomicAdd(A.loss, l * invB);
}

// ------------------------------------------------------------------ backward
// A block of MLP_H threads handles MLP_SPB samples; thread j owns row j of
// dW1 and dW2 and column j of dW3 in LDS, so no LDS atomics are needed;
// the block's sums are added to the global gradients once.
__global__ void __launch_bounds__(MLP_H)
k_mlp_bwd(MlpBwdArgs A) {
    __shared__ float gW1[MLP_H * MLP_IN];
    __shared__ float gW2[MLP_H * MLP_H];
    __shared__ float gW3[MLP_OUT * MLP_H];
    __shared__ float gb1[MLP_H], gb2[MLP_H], gb3[MLP_OUT];
    __shared__ float x[MLP_IN], a1[MLP_H], dz2[MLP_H], dy[MLP_OUT];
    const uint32_t j = threadIdx.x;
    const uint16_t* Wb = A.wbf16;
    for (uint32_t i = j; i < MLP_H * MLP_IN; i += MLP_H) gW1[i] = 0.f;
    for (uint32_t i = j; i < MLP_H * MLP_H; i += MLP_H) gW2[i] = 0.f;
    for (uint32_t i = j; i < MLP_OUT * MLP_H; i += MLP_H) gW3[i] = 0.f;
    gb1[j] = 0.f; gb2[j] = 0.f;
    if (j < MLP_OUT) gb3[j] = 0.f;
    __syncthreads();
    const uint32_t b0 = blockIdx.x * MLP_SPB;
    const uint32_t b1 = min(A.B, b0 + MLP_SPB);
    for (uint32_t b = b0; b < b1; ++b) {
        const float* act = A.act + uint64_t(b) * MLP_ACT;
        for (uint32_t i = j; i < MLP_IN; i += MLP_H) x[i] = A.X[uint64_t(b) * MLP_IN + i];
        a1[j] = act[MLP_H + j];
        if (j < MLP_OUT) dy[j] = A.dY[uint64_t(b) * MLP_OUT + j];
        const float z1 = act[j], z2 = act[2 * MLP_H + j], a2 = act[3 * MLP_H + j];
        __syncthreads();
        // layer 3
        float da2 = 0.f;
        for (int o = 0; o < MLP_OUT; ++o) {
            gW3[o * MLP_H + j] += dy[o] * a2;
            da2 += bf16_to_f32(Wb[MLP_WB_W3 + o * MLP_H + j]) * dy[o];
        }
        if (j < MLP_OUT) gb3[j] += dy[j];
        const float d2 = da2 * gelu_grad_f(z2);
        dz2[j] = d2;
        __syncthreads();
        // layer 2
        for (int k = 0; k < MLP_H; ++k) gW2[j * MLP_H + k] += d2 * a1[k];
        gb2[j] += d2;
        float da1 = 0.f;
        for (int k = 0; k < MLP_H; ++k) da1 += bf16_to_f32(Wb[MLP_WB_W2 + k * MLP_H + j]) * dz2[k];
        const float d1 = da1 * gelu_grad_f(z1);
        // layer 1
        for (int i = 0; i < MLP_IN; ++i) gW1[j * MLP_IN + i] += d1 * x[i];
        gb1[j] += d1;
        __syncthreads();
    }
    float* G = A.grad;
    for (uint32_t i = j; i < MLP_H * MLP_IN; i += MLP_H) atomicAdd(&G[MLP_OFF_W1 + i], gW1[i]);
    for (uint32_t i = j; i < MLP_H * MLP_H; i += MLP_H) atomicAdd(&G[MLP_OFF_W2 + i], gW2[i]);
    for (uint32_t i = j; i < MLP_OUT * MLP_H; i += MLP_H) atomicAdd(&G[MLP_OFF_W3 + i], gW3[i]);
    atomicAdd(&G[MLP_OFF_B1 + j], gb1[j]);
    atomicAdd(&G[MLP_OFF_B2 + j], gb2[j]);
    if (j < MLP_OUT) atomicAdd(&G[MLP_OFF_B3 + j], gb3[j]);
}

// ------------------------------------------------------------------ AdamW
__device__ __forceinline__ int wb_index(uint32_t i) {
    // position of parameter i in the BF16 copy, or -1 for a bias
    if (i < MLP_OFF_B1) return MLP_WB_W1 + (int)(i - MLP_OFF_W1);
    if (i >= MLP_OFF_W2 && i < MLP_OFF_B2) return MLP_WB_W2 + (int)(i - MLP_OFF_W2);
    if (i >= MLP_OFF_W3 && i < MLP_OFF_B3) return MLP_WB_W3 + (int)(i - MLP_OFF_W3);
    return -1;
}

__global__ void k_mlp_adamw(MlpAdamArgs A) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MLP_P) return;
    float* w = A.buf;
    float* g = A.buf + MLP_P;
    float* m = A.buf + 2 * MLP_P;
    float* v = A.buf + 3 * MLP_P;
    const float gi = g[i];
    const float mi = A.beta1 * m[i] + (1.f - A.beta1) * gi;
    const float vi = A.beta2 * v[i] + (1.f - A.beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / A.bc1, vh = vi / A.bc2;
    const float wi = w[i] - A.lr * (mh / (sqrtf(vh) + A.eps) + A.wd * w[i]);
    w[i] = wi;
    g[i] = 0.f;
    const int k = wb_index(i);
    if (k >= 0) A.wbf16[k] = f32_to_bf16(wi);
}

// BF16 copies of the weights from the FP32 masters; gradients cleared.
__global__ void k_mlp_sync(float* buf, uint16_t* wbf16) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MLP_P) return;
    buf[MLP_P + i] = 0.f;
    const int k = wb_index(i);
    if (k >= 0) wbf16[k] = f32_to_bf16(buf[i]);
}

// ------------------------------------------------------------------ sketches
// Histogram of floor(log2 multiplicity) over the keys of a bucketed table.
__global__ void k_deg_hist(const DirEntry* dir, const uint2* pool, uint32_t nbkt, uint32_t* hist) {
    __shared__ uint32_t lh[32];
    if (threadIdx.x < 32) lh[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t j = blockIdx.x;
    if (j < nbkt) {
        const DirEntry e = dir[j];
        const uint32_t cap = 1u << e.log2cap;
        const uint2* base = pool + e.offset;
        for (uint32_t s = threadIdx.x; s < cap; s += blockDim.x) {
            const uint2 kv = base[s];
            if (kv.x != EMPTY_KEY && kv.y) atomicAdd(&lh[31 - __clz(kv.y)], 1u);
        }
        if (threadIdx.x == 0 && e.special) atomicAdd(&lh[31 - __clz(e.special)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 32 && lh[threadIdx.x]) atomicAdd(&hist[threadIdx.x], lh[threadIdx.x]);
}

__global__ void k_sketch_features(const uint32_t* hist3, uint64_t nr, uint64_t ns, uint64_t nt,
                                  int kind, float* f) {
    const uint32_t i = threadIdx.x;
    if (i < 96) f[i] = log2f(1.f + (float)hist3[i]) / 32.f;
    if (i == 96) f[i] = log2f(1.f + (float)nr) / 32.f;
    if (i == 97) f[i] = log2f(1.f + (float)ns) / 32.f;
    if (i == 98) f[i] = log2f(1.f + (float)nt) / 32.f;
    if (i == 99) f[i] = (float)kind;
}

}  // namespace mj
