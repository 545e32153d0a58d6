"""FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library.
"""
from .oracle import (build, load, profile, windows, loglik, elbo,  # noqa: F401
                     log_prior, adam, philox4x32_10, eps_philox,
                     num_threads, profile_asym, windows_asym, elbo_asym,
                     readout, set_threads, profile_sec,
                     windows_sec, elbo_sec)
