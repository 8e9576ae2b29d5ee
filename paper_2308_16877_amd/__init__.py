"""MI355X-native approximated-region library (HPAC-Offload's techniques:
iACT input memoization, TAF output memoization, herded loop perforation).

The compute path is libhpac.so (HIP kernels for gfx950 behind the C ABI in
include/hpac.h); `hpac` is its thin ctypes binding and `inputs` holds the
seeded synthetic input generators.  Build with
`python -m paper_2308_16877_amd.build`.
"""
from .hpac import (hpac_exact, hpac_iact, hpac_taf, hpac_perfo, hpac_probe_copy,  # noqa: F401
                   hpac_bs_vjp, hpac_bs_adjoint, hpac_num_lanes, hpac_trace_entries, hpac_last_error,
                   hpac_abi_version)
