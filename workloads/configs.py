"""The five synthetic workloads used by the tests and the benchmark.

Each stands in for a class of matrices the paper factors (Section 6): the
fractional-Laplacian-like stiffness (s = 0.75) of the headline case, a plain
FP64 case at two sizes, a batch of uneven small instances, and the random
field case that differentiates through the solve.  Seeds are fixed so every
run of every consumer sees the same matrices and right-hand sides.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List

import numpy as np

from .wavelet import WaveletSpec, centers, make_matrix, make_nonsymmetric, mass_spec, normal_rhs


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    spec: WaveletSpec
    nrhs: int
    seed: int          # base seed S; xi uses S, b uses S+1, y* S+2, z S+3, FD choice S+4

    @property
    def n(self) -> int:
        return self.spec.n

    def matrix(self) -> Dict[str, np.ndarray]:
        return make_matrix(self.spec)

    def rhs(self) -> np.ndarray:
        return normal_rhs(self.n, self.nrhs, self.seed + 1)


def small_fp64() -> Workload:
    """64x64 grid, levels 0..5, N = 4096, a = 1.5, exp(-|dc|/0.3) values, one RHS."""
    return Workload("haar64_n4096", WaveletSpec(6, 1.5, 0.5, "exp", 0.3, 1.5, 1000), 1, 1000)


def medium_fp64() -> Workload:
    """256x256 grid, levels 0..7, N = 65536, a = 1.5, one RHS."""
    return Workload("haar256_n65536", WaveletSpec(8, 1.5, 0.5, "exp", 0.3, 1.5, 2000), 1, 2000)


def headline() -> Workload:
    """512x512 grid, levels 0..8, N = 262144, a = 2, s = 0.75, algebraic decay, 64 RHS."""
    return Workload("haar512_n262144_s075", WaveletSpec(9, 2.0, 0.75, "alg", 0.3, 1.75, 3000), 64, 3000)


def random_field() -> Workload:
    """Same operator class as the headline case with its own seed, one RHS."""
    return Workload("haar512_n262144_grf", WaveletSpec(9, 2.0, 0.75, "alg", 0.3, 1.75, 5000), 1, 5000)


def theta_scheme() -> Workload:
    """Time-stepping case (Section 6, parabolic problem for the fractional
    Laplacian): s = 3/8 on the 512x512 Haar grid, one trajectory.  The steps
    use THETA, T_END and NSTEPS below and heat_spot_forcing for f."""
    return Workload("haar512_n262144_s0375_cn", WaveletSpec(9, 2.0, 0.375, "alg", 0.3, 1.75, 6000), 1, 6000)


THETA, T_END, NSTEPS = 0.5, 3.0, 150      # Crank-Nicolson, [0, 3], 150 equidistant steps


def heat_spot_forcing(spec: WaveletSpec, times: np.ndarray) -> np.ndarray:
    """n x len(times) load vectors of a Gaussian heat spot moving on a circle,
    f(x, t) = 100 exp(-40 (x1 - r cos 2 pi t)^2 - 40 (x2 - r sin 2 pi t)^2),
    stand-in for the paper's right-hand side: the grid [0,1]^2 is mapped to
    [-1,1]^2 (the paper's domain is a disc), the circle has radius r = 1/2 so
    the spot stays inside, and the coefficient of a wavelet of level j with
    support centre c is 2^-j f(c, t)."""
    c, level = centers(spec.grid_exp)
    x = 2.0 * c - 1.0
    w = 2.0 ** (-level.astype(np.float64))
    t = np.asarray(times, np.float64)
    px, py = 0.5 * np.cos(2 * np.pi * t), 0.5 * np.sin(2 * np.pi * t)
    d2 = (x[:, 0:1] - px[None, :]) ** 2 + (x[:, 1:2] - py[None, :]) ** 2
    return w[:, None] * 100.0 * np.exp(-40.0 * d2)


def tiny(grid_exp: int, a: float = 1.5, s: float = 0.5, seed: int = 7) -> Workload:
    """Small instances for brute-force checks (N = 4^grid_exp)."""
    return Workload(f"haar{1 << grid_exp}_n{4 ** grid_exp}", WaveletSpec(grid_exp, a, s, "exp", 0.3, 1.5, seed), 1, seed)


def batch_instance(i: int, base_seed: int = 4000) -> Workload:
    """Instance i of the uneven batch: grid side 2^J with J uniform in {5,6,7},
    ell ~ U(0.1,0.5), a ~ U(1.2,2.0), s uniform in {1/4,1/2,3/4}; values as in
    the small case.  The draws come from PCG64(base_seed + 10 + i) in that order."""
    seed = base_seed + 10 + i
    g = np.random.Generator(np.random.PCG64(seed))
    J = int(g.integers(5, 8))
    ell = float(g.uniform(0.1, 0.5))
    a = float(g.uniform(1.2, 2.0))
    s = float(g.choice(np.array([0.25, 0.5, 0.75])))
    return Workload(f"batch{i}_n{4 ** J}", WaveletSpec(J, a, s, "exp", ell, 1.5, seed), 4, seed)


def batch(count: int = 256, base_seed: int = 4000) -> List[Workload]:
    return [batch_instance(i, base_seed) for i in range(count)]


ALL = {
    "small": small_fp64,
    "medium": medium_fp64,
    "headline": headline,
    "grf": random_field,
}


def block_diagonal(mats: List[Dict[str, np.ndarray]]) -> Dict[str, np.ndarray]:
    """The matrices of a batch stacked as diag(A_0, A_1, ...): lower CSC with the
    instances' columns, rows and values in order (rows shifted by the instances
    before), plus seg_ptr, the first unknown of every instance."""
    ns = [int(m["n"]) for m in mats]
    seg = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    zs = np.concatenate([[0], np.cumsum([int(m["colptr"][-1]) for m in mats])]).astype(np.int64)
    colptr = np.concatenate([[0]] + [m["colptr"][1:] + zs[b] for b, m in enumerate(mats)]).astype(np.int64)
    rowind = np.concatenate([m["rowind"] + seg[b] for b, m in enumerate(mats)]).astype(np.int32)
    values = np.concatenate([m["values"] for m in mats])
    return {"n": int(seg[-1]), "colptr": colptr, "rowind": rowind, "values": values, "seg_ptr": seg.astype(np.int32)}


def _instance_matrix(args):
    i, base_seed = args
    return make_matrix(batch_instance(i, base_seed).spec)


def batch_matrices(count: int = 256, base_seed: int = 4000, workers: int = 8) -> List[Dict[str, np.ndarray]]:
    """Matrices of the first count batch instances, generated by a pool of
    forked worker processes (call before any GPU work in the process)."""
    import multiprocessing as mp
    jobs = [(i, base_seed) for i in range(count)]
    if workers <= 1 or count <= 1:
        return [_instance_matrix(j) for j in jobs]
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_instance_matrix, jobs, chunksize=1)


@dataclasses.dataclass(frozen=True)
class PcmLu:
    """Nonsymmetric system on the wavelet pattern, factored by LU (Section 5.1,
    eq:PCM2; Section 6.1 factors A_J by LU on the nested dissection ordering
    of the symmetric pattern)."""
    name: str
    spec: WaveletSpec
    eta: float
    nrhs: int
    seed: int

    @property
    def n(self) -> int:
        return self.spec.n

    def matrix(self) -> Dict[str, np.ndarray]:
        return make_nonsymmetric(self.spec, self.eta, self.seed + 7)

    def rhs(self) -> np.ndarray:
        return normal_rhs(self.n, self.nrhs, self.seed + 1)


def pcm_lu(grid_exp: int = 8, nrhs: int = 8) -> PcmLu:
    """256x256 grid by default (N = 65536, a = 1.5 as the FP64 case), values
    perturbed by up to 50% independently below and above the diagonal; several
    right-hand sides, as the PCM needs many (Section 5.1)."""
    return PcmLu(f"pcm{1 << grid_exp}_n{4 ** grid_exp}_lu", WaveletSpec(grid_exp, 1.5, 0.5, "exp", 0.3, 1.5, 8000),
                 0.5, nrhs, 8000)


@dataclasses.dataclass(frozen=True)
class CovarianceField:
    """Gaussian random field in covariance form (Section 5.3, eq:CholFastField):
    the Galerkin covariance matrix C^G (exponential-type decay with distance,
    standing in for the exp(-|x - x'|) kernel of Section 6.3, whose domain has
    side 4: correlation length 1/4 of the side) and the mass matrix G on the
    same index set, each with its own ordering.  Samples are G^-1 (abar + L X)."""
    name: str
    cov: WaveletSpec
    mass: WaveletSpec
    nsamples: int
    seed: int

    @property
    def n(self) -> int:
        return self.cov.n

    def cov_matrix(self) -> Dict[str, np.ndarray]:
        return make_matrix(self.cov)

    def mass_matrix(self) -> Dict[str, np.ndarray]:
        return make_matrix(self.mass)

    def noise(self, k: int = None) -> np.ndarray:
        return normal_rhs(self.n, self.nsamples if k is None else k, self.seed + 3)

    def mean(self) -> np.ndarray:
        """abar^G: the Galerkin projection of a smooth mean field, here
        sin(2 pi x1) cos(2 pi x2) at the support centres, weighted by 2^-j."""
        c, level = centers(self.cov.grid_exp)
        return np.sin(2 * np.pi * c[:, 0]) * np.cos(2 * np.pi * c[:, 1]) * 2.0 ** (-level.astype(np.float64))


def covariance_field(grid_exp: int = 9, nsamples: int = 64) -> CovarianceField:
    """512x512 grid by default (N = 262144): C^G with a = 2, s = 1/2,
    exp(-|dc| / 0.25) decay; G the mass-matrix stand-in (supports that touch)."""
    return CovarianceField(f"field{1 << grid_exp}_n{4 ** grid_exp}",
                           WaveletSpec(grid_exp, 2.0, 0.5, "exp", 0.25, 1.5, 7000), mass_spec(grid_exp, 7001),
                           nsamples, 7000)
