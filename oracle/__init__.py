"""FP64 CPU oracle for batched TabNet inference -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import, call
or execute anything in this package.  The product path (the HIP library and its
Python binding) never does, and the two share no code: the oracle reads the raw model
parameters and the raw inputs and nothing the HIP path builds.

Modules:
  sparsemax -- sort-based sparsemax plus brute-force-support and bisection references
  rounding  -- bfloat16 / float8-E4M3FN round-to-nearest-even, from the formats' definitions
  tabnet    -- the vectorised float64 TabNet forward (optionally on rounded operands)
  scalar    -- a per-row pure-Python spelling of the same forward, to pin the first
  stats     -- per-feature mean and population variance of masks over a set of rows
  embed     -- categorical embedding of raw rows and the per-raw-column view of the masks
  parallel  -- runs a function of the oracle over row chunks in single-threaded worker
               processes (rows are independent at inference), for full-batch checks

Every function's pin lives in tests/ (marked not-gpu); none is "parity unpinned".
"""
from .sparsemax import sparsemax, sparsemax_tau, sparsemax_support, sparsemax_bisect  # noqa: F401
from .rounding import round_bf16, round_e4m3  # noqa: F401
from .tabnet import forward  # noqa: F401
from .stats import column_mean_var, window_mean_var  # noqa: F401
from .embed import reduce_columns, forward_raw  # noqa: F401
