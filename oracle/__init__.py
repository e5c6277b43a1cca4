"""FP64 CPU oracle for the randomized (H-)Tucker path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package; only ``tests/``, the smoke check and the CPU-baseline
leg of the benchmark do.  It is a plain, slow, obviously correct NumPy
implementation written from the paper, sharing no code with the HIP
library.  Each function cites the passage of the paper it follows.

Conventions (the paper leaves the unfolding order open, Section 2.2): all
tensors are C-ordered, the column index of a mode-k unfolding is the
C-order linear index of the remaining modes in increasing mode order, and
the rows of a multi-mode unfolding X^(S) are C-ordered over the modes of S.

Pins: every function is checked in ``tests/test_oracle_*.py`` against
closed forms, invariants, brute force or the paper's printed facts, except
the sampled-sketch error bound of Theorem 3.4 beyond its exact-rank and
dense special cases, and the randomized H-Tucker beyond exact recovery and
its dense reduction to deterministic RtL-HT (parity unpinned against
theory: the paper gives no bound for it).
"""
from .tensor import unfold, fold, unfold_set, ttm, multi_ttm  # noqa: F401
from .tucker import (gather_fibers, range_sketch, orth, w_step, sub_r_hosvd,  # noqa: F401
                     core, core_streamed, core_chunked, reconstruct, rel_error, mode_errors,
                     projector_distance, canonical_signs, sq_norm, rel_error_orthonormal)
from .htucker import (sub_r_rtl_ht, transfer_tensor, root_transfer, ht_full, ht_bases,  # noqa: F401
                      ht_rel_error, gather_node, kron_cols, ht_full_vjp,
                      ht_residuals_streamed)
from .grads import core_vjp, reconstruct_vjp, loss_and_grads  # noqa: F401
from .sampling import philox4x64_10, draw_indices, draw_omega, box_muller  # noqa: F401
from .brute import (t_hosvd, rtl_ht, unfolding_tail, lower_bound_sq, rhosvd_factor,  # noqa: F401
                    rangefinder_factor, thm34_factor, sampling_event, ht_tails_sq)
