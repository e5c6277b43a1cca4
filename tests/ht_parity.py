"""The tolerance of the H-Tucker error comparison (oracle-side only).

The tolerances on the relative error are stated relative to the oracle's own
error (1e-10 for FP64 arithmetic).  Randomized H-Tucker on a tensor whose
node sketches are numerically rank-deficient determines its kept subspaces
only to the conditioning of the W step, so the oracle's error is itself
determined only to the spread that a perturbation of its inputs at the unit
roundoff produces (a backward-stable computation is exact for such inputs).
`eps_spread` measures that spread with the oracle: it reruns Algorithm 2
with every Gaussian test matrix scaled entry-wise by (1 +- 2^-52), random
signs, and returns the largest change of the relative error.  The GPU result
is then gated at tol * eps_oracle + SPREAD_FACTOR * spread.
"""
import numpy as np

import oracle
import synthgen

SPREAD_FACTOR = 4.0


def eps_spread(X64, tree, ranks, sketches, eps_or, reps=3, seed=0):
    rng = np.random.default_rng(seed)
    spread = 0.0
    for _ in range(reps):
        pert = {}
        for t, sk in sketches.items():
            signs = rng.choice([-1.0, 1.0], sk.omega.shape)
            pert[t] = synthgen.Sketch(sk.idx, sk.omega * (1.0 + 2.0 ** -52 * signs), "f64")
        U, B, _ = oracle.sub_r_rtl_ht(X64, tree, ranks, pert)
        spread = max(spread, abs(oracle.ht_rel_error(X64, tree, U, B) - eps_or))
    return spread


def eps_gate(eps_or, spread, tol):
    return tol * eps_or + SPREAD_FACTOR * spread
