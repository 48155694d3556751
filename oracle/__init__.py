"""Reference oracle for the dedispersion + single-pulse search hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product (the HIP library, its C ABI
or the Python binding) imports, links or calls this package; only the tests,
the smoke check and the CPU-baseline leg of the benchmark do. It is a plain,
slow, obviously-correct CPU implementation in numpy: integer sums are exact
(int64 / uint64 / Python ints) and every floating-point step is FP64.

It follows, in order:
  * Chapter 1, Eq. (1): the cold-plasma dispersion delay between two radio
    frequencies, proportional to DM times the difference of inverse squared
    frequencies;
  * Section 3.2: brute-force incoherent dedispersion (every trial DM sums all
    m channels over N time bins, O(m x N) per trial) and downsampling by a
    user-given factor;
  * Section 2.1: dedispersion over a large set of trial DMs, then a
    single-pulse search by time-domain boxcar filtering that reports
    statistically significant pulses above a user-given threshold.

The paper fixes no rounding, reference frequency, S/N normalisation, boxcar
index or candidate definition; the readings used here are listed in the
module docstring of oracle.dedisp.
"""
from .dedisp import *  # noqa: F401,F403
from .dedisp import __all__  # noqa: F401
