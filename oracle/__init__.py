"""CPU oracle for the compact ADER-HWENO step (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It wraps ``libhwe_oracle.so`` (plain FP64 C++, see
``hwe_oracle.cpp``) through ctypes and shares no code with the GPU library.
"""
from .oracle import OracleMesh, build_oracle, lax_wendroff, llf_flux, spectral_radius, OPTS_DEFAULT  # noqa: F401
