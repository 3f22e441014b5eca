"""MI355X-native multiway hash joins (arXiv 1905.13376): linear and cyclic
three-way joins and the binary cascade, behind the C ABI of ``libmj.so``.

Importing the package loads the HIP library; it fails loudly when the
library is missing (there is no CPU path)."""
from ._lib import (ALGO_3WAY, ALGO_CASCADE, ALGO_ORIENTED, ALGO_SLARGE, ALGO_STAR, ALGO_STAR_CASCADE,  # noqa: F401
                   LINEAR, PLAN_DENSE_KEYS, PLAN_NO_DENSE, PLAN_SYMMETRIC_SIMPLE, TRIANGLE,
                   Context, MJError,
                   Plan, Rel, as_u64, cost_model, rel, slarge_buckets, status_str, LIB_PATH)
