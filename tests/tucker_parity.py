"""The tolerance of the FP64 Tucker error comparison (oracle-side only).

The FP64 gate on the relative error is 1e-10 of the oracle's own error.  On a
low-noise tensor (relative error ~3e-6 at 64^3) the kept subspaces of the W
step (Algorithm 1) are determined only to the conditioning of the sketch, so
the oracle's error itself moves by several 1e-11 of its value when its
Gaussian test matrices are perturbed at the unit roundoff (a backward-stable
computation is exact for such inputs).  `eps_spread` measures that spread:
it reruns Algorithm 1 with every test matrix scaled entry-wise by
(1 +- 2^-52), random signs, and returns the largest change of the relative
error.  The GPU result is gated at tol * eps_oracle + SPREAD_FACTOR * spread,
as the H-Tucker comparison is.
"""
import numpy as np

import oracle
import synthgen

SPREAD_FACTOR = 4.0


def eps_spread(X64, ranks, sketches, eps_or, core_factor="U", reps=3, seed=0):
    rng = np.random.default_rng(seed)
    spread = 0.0
    for _ in range(reps):
        pert = [synthgen.Sketch(s.idx, s.omega * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], s.omega.shape)),
                                "f64") for s in sketches]
        G, U, Q, _, _ = oracle.sub_r_hosvd(X64, ranks, pert, core_factor=core_factor)
        F = U if core_factor == "U" else Q
        spread = max(spread, abs(oracle.rel_error(X64, G, F) - eps_or))
    return spread


def eps_gate(eps_or, spread, tol):
    return tol * eps_or + SPREAD_FACTOR * spread
