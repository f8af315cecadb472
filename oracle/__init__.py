"""TEST INFRASTRUCTURE: the plain CPU oracle and its ctypes binding.

Only tests/, the smoke check and the benchmark's CPU-baseline leg use this
package. It shares no code with the HIP library in paper_2505_00097_amd/.
"""
from .oracle import *  # noqa: F401,F403
