"""The five synthetic workloads of the randomized (H-)Tucker path.

Each config fixes shapes, ranks, decay, relative noise, oversampling and the
number of sampled fibers.  Sizes marked ``full`` are the measured
workloads; ``small`` variants keep the same structure at sizes the FP64
oracle finishes in seconds (used by parity tests).
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class TuckerConfig:
    name: str
    cfg_id: int
    dims: tuple
    ranks: tuple
    decay: float
    noise: float
    p: int
    alpha: int          # s_k = min(alpha * n_k, n_{!=k})
    dtype: str


C1 = TuckerConfig("c1_fp64_64x64x64", 1, (64, 64, 64), (8, 8, 8), 0.5, 1e-6, 5, 10, "f64")
C2 = TuckerConfig("c2_fp32_256^4", 2, (256,) * 4, (32,) * 4, 0.8, 1e-4, 10, 10, "f32")
C3 = TuckerConfig("c3_bf16_40^6", 3, (40,) * 6, (10,) * 6, 0.7, 1e-3, 6, 10, "bf16")

# structurally identical, oracle-sized stand-ins (several tiles plus ragged tails)
C2_SMALL = TuckerConfig("c2_fp32_72x80x96x64", 2, (72, 80, 96, 64), (12, 12, 12, 12), 0.8, 1e-4,
                        10, 10, "f32")
C3_SMALL = TuckerConfig("c3_bf16_24^5x20", 3, (24, 24, 24, 24, 24, 20), (6,) * 6, 0.7, 1e-3, 6,
                        10, "bf16")


@dataclass(frozen=True)
class HTConfig:
    name: str
    cfg_id: int
    n: int
    order: int
    rank: int
    noise: float
    p: int
    w_alpha: int        # w_S = min(w_alpha * n, n_{not in S})
    dtype: str
    # "n": the rule above (parallel tests, Section 4.2.2); "nS": w_S =
    # min(w_alpha^(d-2) n_S, n_{not in S}) (serial tests, Section 4.2.1)
    sample_rule: str = "n"


C5 = HTConfig("c5_ht_fp32_18^8", 5, 18, 8, 12, 1e-5, 4, 20, "f32")
C5_SMALL = HTConfig("c5_ht_fp32_6^8", 5, 6, 8, 4, 1e-5, 4, 20, "f32")
# closed-form 1/||x|| on [1, 15]^8 (H-Tucker serial tests, Section 4.2.1): rank 7,
# w_S = min(20 n, n_notS) fibers per node as in the parallel tests (Section 4.2.2)
C6 = HTConfig("c6_inverse_norm_fp32_15^8", 6, 15, 8, 7, 0.0, 4, 20, "f32")
# the same tensor with the serial tests' rule at alpha = 2: the root's two
# children (n_S = 15^4 = n_notS) are sampled densely
C7 = HTConfig("c7_inverse_norm_fp32_15^8_serial_rule", 7, 15, 8, 7, 0.0, 4, 2, "f32", "nS")

C4_COUNT = 512
C4_CFG_ID = 4

# uneven modes with the shape of the paper's meteorological tensor (Section
# 3.3.2) and its truncation ranks; synthetic values.  The core decays slowly
# (0.97 per index) so that the 150th direction of the last mode stays far
# above the noise; ell = min(r + p, n) caps the first mode at n_1 = 5 and
# widens the last to 160
C8 = TuckerConfig("c8_uneven_fp32_5x10x12x112x80x270", 8, (5, 10, 12, 112, 80, 270),
                  (5, 8, 10, 28, 50, 150), 0.97, 1e-4, 10, 10, "f32")
# oracle-sized stand-in: the same caps, a last mode of ell = 90
C8_SMALL = TuckerConfig("c8_uneven_fp32_5x6x8x20x16x96", 8, (5, 6, 8, 20, 16, 96),
                        (5, 6, 8, 12, 12, 80), 0.97, 1e-4, 10, 10, "f32")
