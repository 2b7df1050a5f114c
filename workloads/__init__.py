"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark."""
from .wavelet import (WaveletSpec, make_matrix, normal_rhs, full_nnz, centers, basis, pair_uniform, splitmix64,
                      make_nonsymmetric, mass_spec)
from .configs import (Workload, small_fp64, medium_fp64, headline, random_field, tiny, batch, batch_instance,
                      block_diagonal, batch_matrices, theta_scheme, heat_spot_forcing, THETA, T_END, NSTEPS,
                      pcm_lu, covariance_field, CovarianceField)
