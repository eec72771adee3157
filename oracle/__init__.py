"""FP64 CPU oracle for the CP stochastic-gradient method (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  It is a plain, slow, obviously correct numpy
implementation of what the HIP library computes, written from the paper
(Yu & Li, "A block-randomized stochastic method with importance sampling
for CP tensor decomposition"), and shares no code with the library.
"""

from . import philox  # noqa: F401
from .cpd import *  # noqa: F401,F403
from .cpd import (ADAGRAD, DECREASING, EUCLIDEAN, FIXED, LEVERAGE, UNIFORM,  # noqa: F401
                  Degenerate, Oracle, RankDeficient)
