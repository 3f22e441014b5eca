/*
 * mj.h -- C ABI of libmj, the MI355X (gfx950) multiway hash-join library.
 *
 * The operations follow the relational statement of Olukotun, Prabhakar,
 * Singhal, Ullman, Zhang, "Efficient Multiway Hash Join on Reconfigurable
 * Hardware" (arXiv 1905.13376):
 *   - linear three-way join  R(A,B) |x| S(B,C) |x| T(C,D)      (Sec. 3, Sec. 4)
 *   - cyclic three-way join  R(A,B) |x| S(B,C) |x| T(C,A)      (Sec. 5)
 *   - the cascade of two binary hash joins, materialising I = R |x| S (Sec. 6.3)
 * Relations are bags: duplicate tuples count with their multiplicity
 * (Example 1's footnote).  The final result is aggregated by COUNT instead
 * of being materialised (Sec. 6, introduction and Sec. 6.3.1).
 *
 * Conventions shared by every entry point
 *   - Keys are 32-bit values compared by bit pattern (int32 or uint32).
 *   - A relation is given by two device column pointers and an element
 *     stride: tuple i is (col0[i*stride], col1[i*stride]).  A row-major
 *     [n, 2] array is col0 = base, col1 = base + 1, stride = 2.
 *   - Every pointer passed to a count call is DEVICE memory owned by the
 *     caller; the library allocates no device memory and keeps no pointer
 *     after a call returns.  The caller supplies a workspace of at least
 *     mj_plan_t.workspace_bytes bytes (256-byte aligned), and mj_plan a
 *     planning workspace of mj_plan_workspace() bytes.
 *   - Count calls are asynchronous on the given HIP stream (a hipStream_t
 *     passed as void*; NULL = the default stream); results are valid after
 *     the stream synchronises.  A context is used by one host thread at a
 *     time (its profiling state, tuning cache and a batch's recording of
 *     launches are not locked): threads that call concurrently need a
 *     context each.  Overlapping calls that share a workspace race.
 *   - Every function returns an mj_status; on an error no kernel has been
 *     launched and outputs are untouched.  No C++ exception crosses the ABI.
 *   - n = 0 is valid and yields zero counts.
 */
#ifndef MJ_H
#define MJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MJ_OK = 0,
    MJ_ERR_INVALID_ARG = -1,   /* NULL pointer, stride < 1, n >= 2^32, bad plan field */
    MJ_ERR_KEY_RANGE = -2,     /* some A value >= a_domain (found by mj_plan)         */
    MJ_ERR_WORKSPACE = -3,     /* workspace smaller than the plan requires            */
    MJ_ERR_PLAN_MISMATCH = -4, /* plan made for other relation sizes or another kind  */
    MJ_ERR_HIP = -5,           /* a HIP runtime call failed                           */
    MJ_ERR_OVERFLOW = -6,      /* a count can exceed 2^64 (host bound)                */
    MJ_ERR_UNSUPPORTED = -7
} mj_status;

typedef struct mj_ctx mj_ctx;

/* A relation: two key columns on the device. */
typedef struct {
    const uint32_t* col0;
    const uint32_t* col1;
    uint64_t n;        /* number of tuples, < 2^32 */
    int64_t stride;    /* elements between consecutive tuples, >= 1 */
} mj_rel;

typedef enum { MJ_LINEAR = 0, MJ_TRIANGLE = 1 } mj_kind;
typedef enum {
    MJ_ALGO_3WAY = 0,          /* partitioned three-way join (Sec. 4 / Sec. 5)      */
    MJ_ALGO_CASCADE = 1,       /* cascade of two binary hash joins (Sec. 6.3)       */
    MJ_ALGO_STAR = 2,          /* linear only: star three-way join, R and T         */
                               /* resident, S streamed once (Sec. 6, star join)     */
    MJ_ALGO_STAR_CASCADE = 3,  /* linear only: cascade of two binary star joins     */
    MJ_ALGO_ORIENTED = 4,      /* cyclic only: one symmetric simple relation, each  */
                               /* triangle counted once along degree-ordered edges  */
    MJ_ALGO_SLARGE = 5         /* linear only, S the largest relation (Sec. 4, the  */
                               /* paragraph after Algorithm 1): R split into        */
                               /* 2^log2_nb parts by a hash of B, T into 2^log2_nc  */
                               /* by a hash of C, S into the pairs of parts; each   */
                               /* pair (R_i's per-B sums, T_j's multiplicities in   */
                               /* LDS) meets its partition S_ij once                */
} mj_algo;

/* mj_plan_t.flags bits.  mj_plan sets the properties it finds; the
 * request bits are read from the caller's plan (MJ_PLANNER_FIXED) and kept. */
enum {
    MJ_PLAN_SYMMETRIC_SIMPLE = 1,/* cyclic: R, S and T are one relation (same columns, */
                                 /* stride and size) that is symmetric, without        */
                                 /* duplicate tuples and without loops (a, a)          */
    MJ_PLAN_DENSE_KEYS = 2,      /* linear: every B value of R and S is < b_domain and */
                                 /* every C value of S and T is < c_domain, both small */
                                 /* enough for direct-indexed tables (see below);      */
                                 /* cyclic, with MJ_PLAN_SYMMETRIC_SIMPLE: every       */
                                 /* vertex id is < b_domain (the oriented join's       */
                                 /* degrees by direct index)                           */
    MJ_PLAN_NO_DENSE = 0x100     /* request: keep the hashed tables even when the keys */
                                 /* are dense                                          */
};
typedef enum {
    MJ_PLANNER_ANALYTIC = 0,   /* cost model with measured device constants        */
    MJ_PLANNER_LEARNED = 1,    /* MLP on degree sketches; analytic fallback         */
    MJ_PLANNER_FIXED = 2       /* keep the bucket fields the caller filled in       */
} mj_planner;

/* Execution plan.  The hyper-parameters are the paper's bucket counts
 * (Sec. 3.1: a hash function's name stands for its number of buckets):
 *   linear:   nb = H*h buckets on B, nc = g buckets on C (Sec. 4)
 *   cyclic:   share = least number of buckets on A of a hub list (Sec. 5:
 *             R is split by H(A) x G(B); here G is one list per B value,
 *             and a list is cut into max(share, ceil(len / 4096)) ranges
 *             of A so that every piece fits in one workgroup's LDS)
 * All bucket counts are powers of two, given by their log2.             */
typedef struct {
    int32_t kind;              /* mj_kind                                   */
    int32_t algo;              /* mj_algo chosen                            */
    uint32_t log2_nb;          /* linear: buckets on B                      */
    uint32_t log2_nc;          /* linear: buckets on C                      */
    uint32_t log2_share;       /* cyclic: least buckets on A of a hub list  */
    uint32_t seed;             /* hash seed                                 */
    uint64_t n_r, n_s, n_t;    /* sizes the plan was made for               */
    uint32_t a_domain;         /* linear: length of the per-A output        */
    uint32_t flags;            /* MJ_PLAN_* properties mj_plan found        */
    uint64_t join2_size;       /* |R |x| S| on B, exact when known, else 0  */
    uint64_t workspace_bytes;  /* bytes the count call needs                */
    double est_ms_3way;        /* planner's time estimates (0 = not known)  */
    double est_ms_cascade;
    double pred_log2_join2;    /* learned planner: predicted log2(1 + |R |x| S|) */
    double pred_log2_out;      /* learned planner: predicted log2(1 + |output|)  */
    double est_ms_star;        /* linear: star three-way estimate (0 = not eligible) */
    double est_ms_star_cascade;/* linear: star cascade estimate (0 = not eligible)   */
    uint32_t b_domain;         /* MJ_PLAN_DENSE_KEYS: 1 + largest B value (linear),  */
                               /* 1 + largest vertex id (cyclic)                    */
    uint32_t c_domain;         /* linear, MJ_PLAN_DENSE_KEYS: 1 + largest C value    */
    uint64_t input_fingerprint;/* hash of the three relations' column pointers,     */
                               /* strides and sizes; a count call given other       */
                               /* relations returns MJ_ERR_PLAN_MISMATCH            */
    double est_ms_slarge;      /* linear: S-largest estimate (0 = not eligible)      */
} mj_plan_t;

/* Context: binds the library to a device (the current one if device < 0). */
int mj_ctx_create(int device, mj_ctx** out);
int mj_ctx_destroy(mj_ctx* ctx);

/* Per-kernel timing.  With profiling on, every kernel a call launches is
 * bracketed by HIP events recorded on the call's stream.  mj_ctx_profile_read
 * waits for those events and returns, per kernel name (32-byte slots in
 * `names`), the summed milliseconds and the number of launches since the
 * last read; it returns the number of entries written (or a negative status). */
int mj_ctx_profile(mj_ctx* ctx, int enable);
int mj_ctx_profile_read(mj_ctx* ctx, int max_entries, char* names, double* total_ms,
                        int64_t* launches);

/* Human-readable name of a status code (static string). */
const char* mj_status_str(int status);

/* Plan a join (synchronous on `stream`: it launches statistics kernels
 * over the inputs and waits for them).  Fills *plan (host memory).  With
 * MJ_PLANNER_FIXED the caller's log2_nb / log2_nc / log2_share / seed / algo
 * are kept and only the sizes and workspace are filled in.  For the linear
 * kind it checks that every A value is < a_domain (MJ_ERR_KEY_RANGE).
 * Sec. 4.2 and Sec. 5.2 give the costs the analytic planner compares.
 * plan_ws: device scratch of at least mj_plan_workspace(kind, |R|, |S|, |T|)
 * bytes, owned by the caller and free again when mj_plan returns
 * (MJ_ERR_WORKSPACE when smaller; checked before any launch).  The plan
 * records a fingerprint of R, S and T (pointers, strides, sizes): count
 * calls accept it for those relations only.  The properties it certifies
 * (MJ_PLAN_DENSE_KEYS, MJ_PLAN_SYMMETRIC_SIMPLE) are facts about the data
 * at planning time; a count call that finds them broken on the device
 * writes all ones (UINT64_MAX) to its output instead of a count.        */
uint64_t mj_plan_workspace(int kind, uint64_t n_r, uint64_t n_s, uint64_t n_t);
int mj_plan(mj_ctx* ctx, int kind, const mj_rel* R, const mj_rel* S, const mj_rel* T,
            uint32_t a_domain, int planner, mj_plan_t* plan, void* plan_ws,
            uint64_t plan_ws_bytes, void* stream);

/* Linear three-way join with per-A count (Sec. 4, Algorithm 1; Example 1):
 *   count_per_a[a] = #{ (r,s,t) in R x S x T : r.a = a, r.b = s.b, s.c = t.c }
 * for a in [0, a_domain); T's second column (D) takes no part.
 * count_per_a: device uint64[a_domain], fully overwritten.
 * A plan with algo MJ_ALGO_SLARGE runs the S-largest form of the
 * three-way join (needs a_domain <= 2^24 and log2_nb + log2_nc <= 12).
 * A plan with algo MJ_ALGO_STAR runs the star three-way join (Sec. 6,
 * linear star join: R and T small dimension relations held resident, the
 * fact relation S streamed once and grouped by B); any other algo runs the
 * partitioned three-way join.  The star join is exact at any size; it is
 * fast while R has at most 4096 distinct B values (its per-B sums then live
 * in one workgroup's LDS), and the planner only picks it then.
 * A three-way plan with MJ_PLAN_DENSE_KEYS (mj_plan sets it when the B and
 * C values it finds are below 2^24 and not much sparser than the tuples)
 * keeps T's multiplicities and the per-B sums in arrays indexed by the key
 * itself rather than in hashed tables: the same join, each lookup one read.
 * The plan certifies the key bounds for the data it was made on: a B or C
 * value at or above its bound at count time sets every count to all ones
 * (UINT64_MAX).                                                          */
int mj_linear3_count(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                     uint32_t a_domain, uint64_t* count_per_a, const mj_plan_t* plan,
                     void* workspace, uint64_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * linear three-way join exactly as mj_linear3_count, with the library's own
 * workspace -- one array of mj_linear3_count_static_max_bytes() bytes
 * (128 MiB) per device, part of the library's code object, held by each
 * device the library runs on until the process ends.  The call allocates
 * nothing.  It returns MJ_ERR_WORKSPACE before any launch when the plan's
 * path needs more than that array (the direct-indexed path of about 2^22
 * tuples per relation fits).  Every call on one device uses the same
 * array: calls that overlap on a device (other streams, other host
 * threads, other contexts) race and must be ordered by the caller.       */
uint64_t mj_linear3_count_static_max_bytes(void);
int mj_linear3_count_static(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                            uint32_t a_domain, uint64_t* count_per_a, const mj_plan_t* plan,
                            void* stream);

/* Cyclic three-way join, total count (Sec. 5):
 *   total[0] = #{ (r,s,t) : r.b = s.b, s.c = t.c, t.a = r.a }
 * With R = S = T = the symmetric edge relation of a simple graph this is
 * trace(A^3) = 6 x (number of triangles).  total: device uint64[1].
 * A plan with algo MJ_ALGO_ORIENTED, which mj_plan offers only when it has
 * found MJ_PLAN_SYMMETRIC_SIMPLE, keeps every edge in one direction (from
 * the end of lower degree, ties broken by a hash of the id) and counts each
 * triangle once by intersecting the out-lists of an edge's ends; total is
 * six times that, the same value.  The degrees come from a sort of the
 * first ends, or, when the plan has MJ_PLAN_DENSE_KEYS, from an array
 * indexed by id.  The plan certifies the property for the data it was made
 * on: if at count time the kept edges are not exactly half of them, or a
 * loop, an end without edges of its own or (dense ids) an id at or above
 * b_domain appears, total is set to all ones (UINT64_MAX).               */
int mj_triangle3_count(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                       uint64_t* total, const mj_plan_t* plan,
                       void* workspace, uint64_t workspace_bytes, void* stream);

/* Cascade of binary hash joins (Sec. 6.3): I(A,C) = R |x| S on B is
 * materialised in the workspace (in chunks when it does not fit), then
 * I |x| T is counted.  Same outputs as mj_linear3_count (kind MJ_LINEAR,
 * out = uint64[a_domain]) or mj_triangle3_count (kind MJ_TRIANGLE,
 * out = uint64[1]).  For the linear kind a plan with algo
 * MJ_ALGO_STAR_CASCADE runs the cascade of binary star joins (R resident,
 * S streamed into I, then T resident and I streamed); it needs
 * |R |x| S| <= 2^28 and returns MJ_ERR_UNSUPPORTED otherwise.            */
int mj_cascade2_count(mj_ctx* ctx, int kind, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                      uint32_t a_domain, uint64_t* out, const mj_plan_t* plan,
                      void* workspace, uint64_t workspace_bytes, void* stream);

/* Distinct count of the linear join's D values per A (the footnotes to
 * Example 1 and to Sec. 4's step list: friends of friends of friends per
 * person, estimated with Flajolet-Martin sketches that merge by union):
 *   D(a) = { t.d : r in R, s in S, t in T, r.a = a, r.b = s.b, s.c = t.c }
 *   sketch[a] = uint32[16] bitmaps: every d in D(a) with
 *               h = MurmurHash3's 32-bit finaliser of (d xor seed) sets bit
 *               (trailing zeros of h >> 4, or 28 when h >> 4 = 0) of bitmap
 *               h & 15
 *   est[a]    = 0 for an empty set, else (16 / 0.77351) * 2^(sum over the
 *               bitmaps of their lowest zero bit / 16)
 * sketch: device uint32[a_domain][16], fully overwritten; est: device
 * double[a_domain] or NULL.  A values must be < a_domain (mj_plan checks
 * this for the linear kind); larger ones are skipped.  The workspace size
 * comes from mj_linear3_distinct_workspace.  Sketches are exact functions
 * of the sets, so they do not depend on the order of the work.          */
uint64_t mj_linear3_distinct_workspace(uint64_t n_r, uint64_t n_s, uint64_t n_t, uint32_t a_domain);
int mj_linear3_distinct(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                        uint32_t a_domain, uint32_t seed, uint32_t* sketch, double* est,
                        void* workspace, uint64_t workspace_bytes, void* stream);

/* The linear join with its result written out (the join of Sec. 4; the
 * paper's experiments aggregate the result instead of storing it, Sec. 6):
 * the tuples (a, b, c, d) of R |x| S |x| T, bags, in nested-loop order --
 * R's tuples in R's order; for each, the S tuples with s.b = r.b in S's
 * order; for each of those, the T tuples with t.c = s.c in T's order.
 * out: device uint32[cap][4]; receives the elements at positions
 * [first, first + cap) of that sequence, as many as exist (rows past the
 * end are not touched).  total: device uint64[1], always written with the
 * sequence's length, so a first call with cap = 0 (out may be NULL) sizes
 * the output, and windows of any size can be taken one after another.
 * The workspace size comes from mj_linear3_materialize_workspace.  Keys are
 * arbitrary 32-bit patterns; no a_domain applies.                        */
uint64_t mj_linear3_materialize_workspace(uint64_t n_r, uint64_t n_s, uint64_t n_t);
int mj_linear3_materialize(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                           uint64_t first, uint64_t cap, uint32_t* out, uint64_t* total,
                           void* workspace, uint64_t workspace_bytes, void* stream);

/* A batch of independent joins (many joins of uneven size; Sec. 5 runs the
 * partition triples one after another on one chip, here the joins share
 * it).  Every item carries its relations, its output (uint64[a_domain] or
 * uint64[1], device) and a plan from mj_plan (or the autotuner).  The call
 * first records each join's work as the ordered list of launches its own
 * call would make (partitions, multiplicity tables, sorts, scans, work
 * queues; cascades, star and oriented plans their whole path), then issues
 * the lists together on `stream`: each step launches one kernel once for
 * every join whose next launch it is, as one grid (per-join argument
 * structs and block counts in a table on the device), so the number of
 * launches follows the longest list rather than the number of joins.  The
 * cells of ALL linear 3-way joins then run in one launch, and the groups of
 * ALL cyclic 3-way joins in two persistent launches that pull work items
 * from device queues.  The device argument tables are copied from pinned
 * host memory.  An eager call reuses the context's buffer, and first waits
 * (on the host) until the previous call's copy out of it has run.  A call
 * under stream capture synchronises nothing with the host: its tables get
 * a buffer of their own, kept until mj_ctx_destroy because every replay
 * reads it, so the whole call can be captured in a HIP graph and replayed.
 * Workspace: at least mj_batch_workspace() bytes (each join's own
 * workspace, then the tables; the call fails with MJ_ERR_WORKSPACE when it
 * is short).  mj_batch_workspace records the joins' work on the host to
 * size the tables, allocating nothing on the device.                       */
typedef struct {
    int32_t kind;
    uint32_t a_domain;
    mj_rel R, S, T;
    uint64_t* out;
    mj_plan_t plan;
} mj_batch_item;

uint64_t mj_batch_workspace(const mj_batch_item* items, int n);
int mj_batch_count(mj_ctx* ctx, const mj_batch_item* items, int n, void* workspace,
                   uint64_t workspace_bytes, void* stream);

/* Autotuner: times candidate plans of this join on the device (HIP events
 * on `stream`; synchronous) and keeps the fastest: for the linear kind
 * both algorithms and B / C bucket counts 2^8..2^10, for the cyclic kind
 * the shares 1, 4, 16 (and the cascade when the planner rated it within a
 * factor of 4).  `plan` must come from mj_plan for these relations; it is
 * overwritten with the winner.  Results are cached in the context per size
 * class (log2 of the three sizes and of the intermediate), so a second
 * call on a join of the same class costs no runs.  The workspace must hold
 * the largest candidate (mj_plan's workspace_bytes covers all of them).
 * Counts written to `out` (uint64[a_domain] or uint64[1]) by the runs are
 * those of the final plan.  *tuned_ms receives the winner's time.       */
int mj_autotune(mj_ctx* ctx, int kind, const mj_rel* R, const mj_rel* S, const mj_rel* T,
                uint32_t a_domain, uint64_t* out, mj_plan_t* plan, void* workspace,
                uint64_t workspace_bytes, double* tuned_ms, void* stream);

/* The paper's analytic cost formulas as the planner evaluates them (for
 * inspection and testing): tuples read onto the chip by the linear join
 * (Sec. 4.2), moved by the cascade (Example 3), the break-even capacity of
 * Example 3, the cyclic cost and its optimum (Sec. 5.2), the uniform-key
 * size of a binary join (Sec. 6.3) and the branch probability of App. A.
 * args as listed per formula; *out receives the value.                   */
typedef enum {
    MJ_COST_LINEAR_TUPLES = 0,     /* R, S, T, M          */
    MJ_COST_CASCADE_TUPLES = 1,    /* I                   */
    MJ_COST_LINEAR_BREAK_EVEN_M = 2, /* R, S, T, I        */
    MJ_COST_CYCLIC_TUPLES = 3,     /* R, S, T, M, H       */
    MJ_COST_CYCLIC_OPTIMAL_H = 4,  /* R, S, T, M          */
    MJ_COST_CYCLIC_MIN = 5,        /* R, S, T, M          */
    MJ_COST_JOIN2_UNIFORM = 6,     /* R, S, d             */
    MJ_COST_BRANCH_HIT = 7         /* g3, d               */
} mj_cost_formula;
int mj_cost_model(int which, const double* args, int nargs, double* out);

/* Bucket counts of the S-largest plan (Sec. 4, the paragraph after
 * Algorithm 1) for relations of n_r, n_s, n_t tuples: *log2_nb = log2 L_R
 * (parts of R of about 1024 tuples), *log2_nc = log2 L_T (the count the
 * planner's time model prefers, log2_nb + log2_nc <= 12) and *est_ms the
 * modelled time (may be NULL).  Host only, no device needed.  Returns
 * MJ_ERR_INVALID_ARG for NULL outputs or when R needs more than 2^12
 * parts; the outputs are then left unchanged.                            */
int mj_slarge_buckets(uint64_t n_r, uint64_t n_s, uint64_t n_t, uint32_t* log2_nb, uint32_t* log2_nc,
                      double* est_ms);

/* ---------------------------------------------------------------------
 * Learned planner (not from the paper; its choices never change a count).
 * A join is summarised by a degree sketch of MJ_SKETCH_DIM features: for
 * R's B column, S's B column and T's C column a 32-bin histogram of
 * floor(log2 deg(v)) over their distinct values v (each bin given as
 * log2(1 + keys in the bin) / 32), then log2(1 + |R|), (1 + |S|), (1 + |T|)
 * over 32, then the kind.  A network MJ_SKETCH_DIM -> 64 -> 64 -> 11 with
 * GELU maps it to: predicted log2(1 + |R |x| S|), log2(1 + |output|),
 * logits of the plan in mj_algo order (three-way, cascade, star, star
 * cascade, oriented, S-largest) and of the share (1, 4, 16).  mj_plan
 * takes the plan of largest logit among those the join is eligible for.
 * Weights are BF16 (W1, W2, W3), biases and arithmetic FP32.
 * The parameter buffer is device memory of mj_mlp_param_bytes() bytes:
 *   float master[P], grad[P], adam_m[P], adam_v[P]; uint16 bf16_weights[]
 * with P = 64*100 + 64 + 64*64 + 64 + 11*64 + 11 parameters in the order
 * W1 (row-major [64][100]), b1, W2 ([64][64]), b2, W3 ([11][64]), b3.
 * All calls are asynchronous on `stream` and launch kernels only.       */
#define MJ_SKETCH_DIM 100
#define MJ_MLP_HIDDEN 64
#define MJ_MLP_OUT 11
uint64_t mj_mlp_param_bytes(void);
/* BF16 copies from the FP32 masters; gradients cleared. */
int mj_mlp_sync(mj_ctx* ctx, void* params, void* stream);
/* Y[B][11] = network(X[B][100]) (device fp32 arrays). */
int mj_mlp_forward(mj_ctx* ctx, const void* params, const float* X, uint32_t B, float* Y,
                   void* stream);
/* Forward, loss and backward of a batch: the gradients are ADDED to the
 * grad block of `params`; *loss (device fp32) is increased by the batch's
 * mean loss: squared error of heads 0-1 against targets[B][2], softmax
 * cross entropy of heads 2-7 against plan_label[B] (an mj_algo value,
 * 0..5) and of heads 8-10 against share_label[B] (0, 1, 2 for 1, 4, 16;
 * -1 = no share term).  Workspace: mj_mlp_workspace(B).               */
uint64_t mj_mlp_workspace(uint32_t B);
int mj_mlp_grads(mj_ctx* ctx, void* params, const float* X, uint32_t B, const float* targets,
                 const int32_t* plan_label, const int32_t* share_label, float* loss,
                 void* workspace, uint64_t workspace_bytes, void* stream);
/* One AdamW step (beta 0.9 / 0.999, eps 1e-8, decoupled weight decay) at
 * step number `step` (>= 1); refreshes the BF16 copies, clears gradients. */
int mj_mlp_adamw(mj_ctx* ctx, void* params, float lr, float weight_decay, uint32_t step,
                 void* stream);
/* The degree sketch of a join (features: device fp32[MJ_SKETCH_DIM]). */
uint64_t mj_sketch_workspace(uint64_t n_r, uint64_t n_s, uint64_t n_t);
int mj_sketch(mj_ctx* ctx, int kind, const mj_rel* R, const mj_rel* S, const mj_rel* T,
              float* features, void* workspace, uint64_t workspace_bytes, void* stream);
/* Network used by mj_plan with MJ_PLANNER_LEARNED (NULL: the analytic
 * planner is used instead).  The buffer stays owned by the caller and must
 * live while plans are made. */
int mj_ctx_set_planner(mj_ctx* ctx, const void* params);

/* Exact |R |x| S| on B = sum_b deg_R(b) * deg_S(b) (the cascade's
 * intermediate size, Sec. 6.3), computed on the device.  Synchronous;
 * *out is host memory.  Needs a workspace of mj_join2_size_workspace()
 * bytes.                                                                 */
uint64_t mj_join2_size_workspace(uint64_t n_r, uint64_t n_s);
int mj_join2_size(mj_ctx* ctx, const mj_rel* R, const mj_rel* S, uint64_t* out,
                  void* workspace, uint64_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MJ_H */
