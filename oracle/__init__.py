"""Plain FP64 CPU oracle for JK-CALS (arXiv 2112.03985).

TEST INFRASTRUCTURE ONLY.  The only code allowed to import, call or run
anything in this package is the test suite, the smoke check of the HIP path,
and the CPU-baseline leg of the benchmark.  The product path (the HIP library
and its Python binding) never routes through it, and this package imports
nothing from the product.

What it computes, and from which passage:

* ``cp``        -- the building blocks of CP-ALS (Sec. 3.2, Alg. 1): mode-n
                   unfolding (Eq. (3)), Khatri-Rao product in the order of
                   Eq. (1), MTTKRP, Hadamard product of Gramians, the
                   normal-equation update, the error identity.
* ``jackknife`` -- leave-one-out jackknife by fitting every submodel on its
                   explicitly reduced tensor (Alg. 2, the slice removal and
                   row removal steps followed by CP-ALS), per-iteration
                   records, the CP least-squares loss and its gradient, the
                   gradient-refinement rule, and the flop counts of Sec. 4.2.
* ``postprocess`` -- the end of Alg. 2: permutation and scale adjustment of
                   every submodel against the overall model, and the
                   standard deviation of the factors over the submodels.

JK-CALS (Alg. 3) changes performance, not the numerics: by Case I and
Case II of Sec. 4.1 its fused MTTKRP equals each submodel's own MTTKRP on the
reduced tensor, and its Hadamard/update steps stay per submodel.  So the
oracle is the plain per-submodel ALS, written with no fusion, no blocking and
no padding tricks, in float64.

Readings of passages that are silent or garbled (each repeated where used):

* error identity: the sign in front of the Hadamard-of-Gram term is taken as
  "+" (the identity the paper cites; the printed "-" cannot hold at an ALS
  fixed point);
* pseudoinverse update: Cholesky when H is positive definite, otherwise an
  eigen-decomposition pseudoinverse with cutoff R*eps*lambda_max(H);
* normalisation: after every mode update the columns are scaled to unit
  2-norm and the norms kept as lambda (absent from the paper, standard
  practice, does not change the fitted model);
* fit = 1 - ||T - [[lambda; U]]|| / ||T||, convergence when |delta fit| < tol;
* Gram matrices are made exactly symmetric by mirroring the upper triangle;
* jackknife post-processing: matching by the product over the non-sampled
  modes of the column cosines (exact assignment), unit-norm columns with
  signs aligned to the reference, and the jackknife standard deviation
  sqrt((K-1)/K * sum (theta - mean)^2).

Parity status of each function is stated in its docstring; the pins that tie
it to the paper and to mathematics live in ``tests/test_oracle_*.py``.
"""
from .cp import (unfold, khatri_rao, krp_excluding, mttkrp, mttkrp_bruteforce,
                 gram, hadamard_of_grams, solve_normal, normalise_columns,
                 error_fast, reconstruct, residual_explicit)
from .jackknife import (reduce_tensor, reduce_init, left_out_rows, cp_als, jk_als, loss, grad,
                        loss_and_grad, fd_grad, gd_refine, flops_jk_als,
                        flops_jk_cals, flop_ratio, model_offsets, ModelResult)
from .postprocess import congruence, match_components, aligned_factors, jackknife_std

__all__ = [
    "unfold", "khatri_rao", "krp_excluding", "mttkrp", "mttkrp_bruteforce",
    "gram", "hadamard_of_grams", "solve_normal", "normalise_columns",
    "error_fast", "reconstruct", "residual_explicit", "reduce_tensor",
    "reduce_init", "left_out_rows", "cp_als", "jk_als", "loss", "grad", "loss_and_grad", "fd_grad",
    "gd_refine", "flops_jk_als", "flops_jk_cals", "flop_ratio", "model_offsets",
    "ModelResult", "congruence", "match_components", "aligned_factors", "jackknife_std",
]
