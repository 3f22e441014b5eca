// Host-side helpers of libmj shared by the API translation units (internal).
#pragma once
#include <stdint.h>

#include "mj.h"

namespace mj {

int check_rel(const mj_rel* r);
uint32_t ceil_log2(uint64_t x);
uint32_t join2_bits(uint64_t n);
int plan_workspace(mj_plan_t& p);

}  // namespace mj
