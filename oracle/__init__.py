"""FP64 CPU oracle for the FFT-based Core-AFD loop (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg import this
package; the product path never does.
"""
from .afd_oracle import *  # noqa: F401,F403
from .afd_oracle import __all__  # noqa: F401
