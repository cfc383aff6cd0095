"""FP64 CPU oracle for entropic optimal transport by Sinkhorn-Knopp and
SK-NR(l).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that
the GPU path is checked against.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product library
never calls it and shares no code with it.

Everything here is float64 numpy, written to be read against the paper
(Chhaibi, Gratton, Vaiter, "Faster Computation of Entropic Optimal
Transport via Stable Low Frequency Modes", arXiv 2506.14780).  Each
function cites the section / equation / algorithm it follows.
"""
from .sk import *  # noqa: F401,F403
from .sk import __all__  # noqa: F401
