"""FP64 CPU oracle for the TV-model EM hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct numpy/scipy implementation of what one
augmented-formulation TV-model EM iteration computes (Vestman et al., 2019):
full-covariance UBM frame posteriors, Baum-Welch statistics, the E-step of
eqs. (3)-(4), the M-step accumulators, the M-step solve of the cited
factor-analysis EM, minimum-divergence re-estimation (eqs. (6)-(12)) and the
UBM-mean realignment of Sec. 3.2.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path
and imports nothing from it; the product path never calls it.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
against something other than itself (brute-force densities, Gaussian
conditioning of the joint, brute-force marginal likelihoods, finite
differences of the EM auxiliary function, stated invariants).  The one
learned-selection functions of ``mlp`` are pinned by finite differences,
closed forms and the k = C special case.  The scoring back-end of ``backend``
(whitening, length normalisation, LDA, two-covariance PLDA, EER) is pinned
by closed forms, quadrature, brute force and invariants.
"""
from .tv import (  # noqa: F401
    LOG2PI,
    frame_loglik,
    posteriors,
    bw_stats,
    init_tv,
    tv_precompute,
    estep,
    accumulate,
    objective,
    mstep,
    mindiv,
    realign_means,
    extract,
    em_iteration,
    diag_frame_loglik,
    preselect,
    pruned_posteriors,
    init_tv_standard,
    center_stats,
    mindiv_standard,
    em_iteration_standard,
)
from .mlp import (  # noqa: F401
    feature_stats,
    standardise,
    mlp_forward,
    round_bf16,
    mlp_forward_bf16,
    log_softmax,
    softmax,
    ce_loss,
    mlp_backward,
    adam_update,
    topk,
    proposed_mass,
    learned_posteriors,
    missed_mass,
)
from . import backend  # noqa: F401,E402
