"""FP64 CPU oracle for the per-pixel chain statistics and the regional reconstruction filter.

TEST INFRASTRUCTURE, NOT PRODUCT CODE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It shares no code with the HIP
path (``paper_2402_08273_amd``) and imports nothing from it.

Everything here is a plain, literal float64 NumPy transcription of the definitions, written
for a reader to check against the paper by eye:

* :mod:`oracle.chain_stats`  -- Appendix A (Correlation and Convergence): the estimator mean,
  the sample variance, lag autocovariances, autocorrelations and the autocorrelation time,
  applied to each pixel's sample sequence;
* :mod:`oracle.regional_filter` -- the reconstruction filter h_j of the path integral
  (Sec. 3.1, eq. path_integral) with its width taken from the per-region parameter
  lambda_k = log sigma_k^2 (Sec. 5.3, "Updating the Scaling Parameter") through the
  state-dependent lookup of Sec. 5.2 on the N x N screen grid of Sec. 6.1; its adjoint;
  and the MSE loss used to drive the adjoint;
* :mod:`oracle.region_adapt` -- the regional adaptation of lambda_k from a stream of
  (region, acceptance probability) proposals: Algorithm 1 with eqs. est_exp_acc,
  update_lambda and step_size_n, one proposal at a time;
* :mod:`oracle.quadtree` -- quadtree partitions (a forest: one tree for the screen, one per
  top-level grid cell for the 4-D partition), leaf lookup and the counting-based refinement
  of Sec. 6.1-6.3, pointer-based;
* :mod:`oracle.direction_sampler` -- the perturbation of a ray direction (Sec. 3.3): the
  polar angle from the normal truncated to [-pi, pi] by its inverse CDF, with sigma_k from
  lambda_k, the azimuth uniform, in the Duff et al. (2017) frame;
* :mod:`oracle.rrmse` -- the relative root-mean-square error of an image against a
  reference, per pixel and for the image (Sec. 8.2);
* :mod:`oracle.lens_chain` -- one Metropolis step of screen-space chains under the regional
  adaptive lens perturbation (Sec. 3.3, Sec. 6.1, Alg. 1 lines 8-13), with an image's
  luminance standing in for the path contribution.

Parity status: every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` (brute force on tiny inputs, exact rational examples, closed forms
of seeded distributions, invariants, finite differences).
"""

from .chain_stats import (  # noqa: F401
    pixel_moments,
    lag_autocovariances,
    chain_statistics,
    stats_accumulate,
)
from .regional_filter import (  # noqa: F401
    LAMBDA_MIN_DEFAULT,
    N_REGIONS_DEFAULT,
    region_index,
    region_sigma_sq,
    filter_forward,
    mse_loss_seed,
    filter_backward,
)
from . import direction_sampler, lens_chain, quadtree, region_adapt, rrmse  # noqa: F401
