"""MI355X-native hot path of the GW polarizability step (BerkeleyGW paper).

Pair densities M_vc(G) by batched FP64 3D FFTs, the chi-sum
chi0 = M^H diag(w) M on MFMA (FP64, or split BF16 with FP32 accumulation
and FP64 recombination), and epsilon = 1 - v chi0 with its FP64 inversion,
all as hand-written HIP kernels for gfx950 behind the C-ABI in
``include/bgw.h``.  Importing this package loads nothing; the native
library is loaded on first use by :mod:`paper_1111_4429_amd.bgw`.
"""

__all__ = ["synth", "bgw"]
