"""FP64 CPU oracle for KK (far-field compressive) plane-wave beamforming.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute
anything in this package: only the tests, the package's smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP library.

It is a plain, slow, step-by-step FP64 statement of what the method computes
(Khetan & Mertz, "Far-field compressive ultrasound beamforming"):

  geometry.py    element positions, transmit angles, image grid (Sec. II-A/B)
  selection.py   receive-angle sets and (tx, rx, set) pairs: Eq. 6, Eq. 7, same-angle,
                 uniform bank; compression L/(J M) (Sec. II-C, II-D)
  luts.py        separable delay tables LUT1..LUT4 and the DAS receive table
                 (Sec. II-F), integer shear table for Eq. 3
  spectrum.py    analytic (Hilbert) spectrum and inverse transform (Sec. II-F)
  decompose.py   Eq. 3 receive plane-wave decomposition by the Fourier shift theorem
  beamform.py    Eq. 5 (KK) and Eq. 4 (DAS) delay-gather sums
  compound.py    Eq. 8 / Eq. 9 compounding, |B|^2
  completion.py  the k-space completion network on the per-bin pair grid (convolutions,
                 gradients, masked loss, Adam, grid preparation and merge); imported as
                 oracle.completion, not re-exported here

Conventions the paper leaves open are fixed in each module's docstring.  Every function
states the passage it follows.  Pins (tests marked "not gpu") check each step against
closed forms, special cases, physics and brute force rather than against itself.
"""
from .geometry import element_positions, tx_angles, grid_axis, next_pow2
from .selection import select_pairs, SHIFTED, CONFOCAL, SAME, FULL_UNIFORM
from .luts import build_luts, das_rx_table, fft_length
from .spectrum import analytic_spectrum, inverse_bins, analytic_signal
from .decompose import decompose, decompose_spectrum
from .beamform import kk_beamform, das_beamform, lerp_gather
from .compound import coherent, incoherent, intensity

__all__ = [
    "element_positions", "tx_angles", "grid_axis", "next_pow2",
    "select_pairs", "SHIFTED", "CONFOCAL", "SAME", "FULL_UNIFORM",
    "build_luts", "das_rx_table", "fft_length",
    "analytic_spectrum", "inverse_bins", "analytic_signal",
    "decompose", "decompose_spectrum", "kk_beamform", "das_beamform", "lerp_gather",
    "coherent", "incoherent", "intensity",
]
