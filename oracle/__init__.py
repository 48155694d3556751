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

  * Section 2.1, before dedispersion: RFI mitigation by bandpass correction
    and time- and frequency-domain flagging, as the figure of the paper's
    RFI tool describes it (oracle.rfi);
  * Sections 2.1 and 3.3: robust noise statistics (sigma-clipped moments,
    median and MAD) for the S/N of the search (oracle.robust);
  * Section 2.1, after the search: removal of redundant candidates of one
    event with square stencils in the DM-time plane, then clustering of the
    candidates in the DM-time plane keeping the highest-S/N one per cluster
    (oracle.sift);
  * Section 3.3: de-reddening of the searched series by running-median
    subtraction (oracle.robust);
  * Section 3.5: the folding transform (FFA) of a series at a base period
    and the boxcar search of the folded profiles (oracle.ffa).

The paper fixes no rounding, reference frequency, S/N normalisation, boxcar
index, candidate definition, stencil size or clustering parameter; the
readings used here are listed in the module docstrings of oracle.dedisp,
oracle.rfi, oracle.robust, oracle.sift and oracle.ffa.
"""
from .dedisp import *  # noqa: F401,F403
from .dedisp import __all__ as _dedisp_all
from .rfi import *  # noqa: F401,F403
from .rfi import __all__ as _rfi_all
from .robust import *  # noqa: F401,F403
from .robust import __all__ as _robust_all
from .sift import *  # noqa: F401,F403
from .sift import __all__ as _sift_all
from .ffa import *  # noqa: F401,F403
from .ffa import __all__ as _ffa_all

__all__ = (list(_dedisp_all) + list(_rfi_all) + list(_robust_all) + list(_sift_all)
           + list(_ffa_all))
