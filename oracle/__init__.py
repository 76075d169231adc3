"""Python access to the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package. The GPU library never imports, links or calls it.
"""
from .oracle import *  # noqa: F401,F403
