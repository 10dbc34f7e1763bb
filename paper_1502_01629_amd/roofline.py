"""Algorithmic work per unit of the hot-path kernels, and MI355X peaks, for roofline reporting.

The counts follow the scheme's definition (Section 3), not the instructions a kernel happens to
execute, so a kernel that evaluates the same formula with fewer instructions shows a higher
achieved rate.

Per foot of a control (one bilinear reconstruction):
  foot offset            2 FMA                 4 flop
  cell fractions         2 sub                 2 flop
  bilinear value         3 x (sub + FMA)       9 flop
                                              15 flop
Per control, on top of its K feet:
  SL2  K-1 adds to sum the feet, 1 max                        K flop
  SL3  K-1 adds (sum), K products (own weight), K-1 adds (Lambda0),
       numerator FMA 2, denominator FMA 2, comparison 3        3K + 5 flop
Per node: the final scaling (SL2 1 mul; SL3 1 mul + 1 div).
Bytes per node-update of a Jacobi sweep: read w 4, write w 4, class 1, speed 4 = 13 B.
"""
from __future__ import annotations

# Published MI355X figures.
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3     # packed/dual-issue FP32 vector peak
FP32_VALU_ISSUE_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s
BF16_MFMA_PEAK_TFLOPS = 2500.0

FEET = {0: 1, 1: 4, 2: 2}


def sweep_flops_per_node_update(diffusion: int, scheme: int, n_controls: int) -> int:
    K = FEET[int(diffusion)]
    per_foot = 15 * K
    if int(scheme) == 0:
        return n_controls * (per_foot + K) + 1
    return n_controls * (per_foot + 3 * K + 5) + 2


SWEEP_BYTES_PER_NODE_UPDATE = 13
