"""Problem instances: grids, wavenumber fields and sources.

Every array here is *input data* of the stochastic Helmholtz problem
-Δu - k(x,ξ)² u = f on the unit interval or square (Section 3), with the random
field written as k(x,ξ) = k_0(x) + Σ_ℓ ξ_ℓ k_ℓ(x), ξ_ℓ ~ U[-1,1] independent
(Section 2.2, eq. random_wavenumber).  Nodes are x_i = i·h, i = 0..n-1 with
h = 1/(n-1) (Appendix A, grids grid_1d / grid_2d, n = q+2); in 2D the node
(x_i, y_j) sits at flat index j·n + i (x fastest, Theorem A.3 ordering).

Readings of points the paper leaves open (stated once here, used by both the
oracle and the GPU path):
  * "Grid with N nodes" counts the boundary nodes, so h = 1/(N-1).
  * A Gaussian source of width w is f(x) = exp(-|x-c|²/(2w²)) (unnormalised).
  * The 2D sine-mode field is k = k̄ + σ Σ_ℓ ℓ⁻¹ sin(a_ℓ π x) sin(b_ℓ π y) ξ_ℓ
    with (a,b) taken in the order MODES; a config with s modes uses the first s.
  * Mesh-size rule of Section 6: lev = max(ceil(log2(15·maxk/(2π))), 1),
    q = 2^lev - 1, where maxk is the *mean* wavenumber k̄ (the printed numbers of
    Section 6 are reproduced only with that reading).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# (a_ℓ, b_ℓ) of the sine modes, ℓ = 1..6.
MODES = [(1, 1), (2, 1), (1, 2), (2, 2), (3, 1), (1, 3)]


@dataclass
class Instance:
    """One stochastic Helmholtz problem with absorbing (or Dirichlet) BC."""

    name: str
    dim: int                 # 1 or 2
    n: int                   # nodes per side (boundary included for absorbing BC)
    s: int                   # number of random variables
    degree: int              # total PC degree r
    k_fields: np.ndarray     # (s+1, n**dim) float64: k_0..k_s at the nodes
    k_mean: float            # spatially constant k_0 (NaN when k_0 varies)
    f: np.ndarray            # (n**dim,) float64 source at the nodes
    bc: str = "absorbing"    # "absorbing" | "dirichlet"
    beta: float = 0.5        # CSL shift β (Section 6 uses β = 1/2)
    restart: int = 50
    tol: float = 1e-8
    meta: dict = field(default_factory=dict)

    @property
    def h(self) -> float:
        return 1.0 / (self.n - 1) if self.bc == "absorbing" else 1.0 / (self.n + 1)

    @property
    def points(self) -> int:
        return self.n ** self.dim

    @property
    def Q(self) -> int:
        return math.comb(self.s + self.degree, self.s)

    @property
    def unknowns(self) -> int:
        return self.Q * self.points


def grid_rule_q(maxk: float) -> int:
    """Number of interior nodes q from the mesh-size rule of Section 6."""
    lev = max(math.ceil(math.log2((15.0 * maxk) / (2.0 * math.pi))), 1)
    return 2 ** lev - 1


def _coords(n: int, dim: int, bc: str = "absorbing"):
    if bc == "absorbing":
        x = np.linspace(0.0, 1.0, n)
    else:  # interior nodes only
        x = np.arange(1, n + 1) / (n + 1)
    if dim == 1:
        return (x,)
    X, Y = np.meshgrid(x, x, indexing="xy")  # X[j, i] = x_i, Y[j, i] = y_j
    return X.ravel(), Y.ravel()


def sine_mode_fields(n: int, kbar: float, sigma: float, s: int) -> np.ndarray:
    """k_0 = k̄ and k_ℓ = σ ℓ⁻¹ sin(a_ℓπx) sin(b_ℓπy) on the n×n node grid."""
    if s > len(MODES):
        raise ValueError("at most %d sine modes are defined" % len(MODES))
    X, Y = _coords(n, 2)
    k = np.empty((s + 1, n * n))
    k[0] = kbar
    for l in range(1, s + 1):
        a, b = MODES[l - 1]
        k[l] = sigma / l * np.sin(a * np.pi * X) * np.sin(b * np.pi * Y)
    return k


def gaussian_source(n: int, dim: int, centre, width: float) -> np.ndarray:
    c = np.atleast_1d(np.asarray(centre, dtype=np.float64))
    xs = _coords(n, dim)
    r2 = sum((xs[d] - c[d]) ** 2 for d in range(dim))
    return np.exp(-r2 / (2.0 * width * width))


def point_source(n: int, dim: int, bc: str = "absorbing") -> np.ndarray:
    """Point source at 1/2 (Appendix A, Point sources): 1/h^dim at node t=ceil(q/2)."""
    if bc == "absorbing":
        q = n - 2
        h = 1.0 / (q + 1)
        t = (q + 1) // 2          # node index on 0..q+1
        idx = t
    else:
        q = n
        h = 1.0 / (q + 1)
        t = (q + 1) // 2          # interior node x_t, stored at position t-1
        idx = t - 1
    f = np.zeros(n ** dim)
    if dim == 1:
        f[idx] = 1.0 / h
    else:
        f[idx * n + idx] = 1.0 / (h * h)
    return f


# ----------------------------------------------------------------- configs

def config1() -> Instance:
    """1D, 201 nodes, k(ξ) = 20 + 2ξ, degree 5 (Q=6), Gaussian at 0.5 width 0.05."""
    n = 201
    k = np.empty((2, n))
    k[0] = 20.0
    k[1] = 2.0
    return Instance("c1_1d_n201_q6", 1, n, 1, 5, k, 20.0,
                    gaussian_source(n, 1, 0.5, 0.05), restart=30, tol=1e-10)


def config2() -> Instance:
    """2D 255², k̄=20, σ=2, s=4, degree 3 (Q=35), Gaussian at the centre."""
    n = 255
    return Instance("c2_2d_n255_q35", 2, n, 4, 3, sine_mode_fields(n, 20.0, 2.0, 4), 20.0,
                    gaussian_source(n, 2, (0.5, 0.5), 0.05), restart=50, tol=1e-8)


def config3() -> Instance:
    """2D 511², k̄=40, σ=4, s=6, degree 3 (Q=84), Gaussian at the centre."""
    n = 511
    return Instance("c3_2d_n511_q84", 2, n, 6, 3, sine_mode_fields(n, 40.0, 4.0, 6), 40.0,
                    gaussian_source(n, 2, (0.5, 0.5), 0.05), restart=50, tol=1e-8)


def small_2d(n: int = 33, kbar: float = 8.0, sigma: float = 0.8, s: int = 2, degree: int = 2,
             centre=(0.5, 0.5), width: float = 0.1, restart: int = 30, tol: float = 1e-10) -> Instance:
    """Down-sized 2D instance of the same family as configs 2 and 3."""
    return Instance("small_2d_n%d_s%d_r%d" % (n, s, degree), 2, n, s, degree,
                    sine_mode_fields(n, kbar, sigma, s), kbar,
                    gaussian_source(n, 2, centre, width), restart=restart, tol=tol)


def degree_sweep_instance(degree: int, n: int = 129, kbar: float = 20.0, sigma: float = 2.0) -> Instance:
    """Constant-mean analogue of the Section 7 degree study (three random variables, 127
    interior nodes per side, point source at the centre, degree 0..8, Q up to 165): sine
    mode fields instead of the wedge, so that the mean block has constant k̄."""
    return Instance("sweep_2d_n%d_s3_r%d" % (n, degree), 2, n, 3, degree, sine_mode_fields(n, kbar, sigma, 3), kbar,
                    point_source(n, 2), restart=200, tol=1e-8)


def config4_instances(count: int = 512, seed0: int = 0) -> list[Instance]:
    """Batched workload: per seed, N∈{63,127,255}, k̄~U[5,30], σ=0.1k̄, s∈{1..4},
    degree∈{2,3,4}, Gaussian (width 0.05) at a uniform point of [0.2,0.8]²."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        n = int(rng.choice([63, 127, 255]))
        kbar = float(rng.uniform(5.0, 30.0))
        s = int(rng.integers(1, 5))
        degree = int(rng.integers(2, 5))
        c = rng.uniform(0.2, 0.8, size=2)
        out.append(Instance("c4_%03d" % (seed0 + i), 2, n, s, degree,
                            sine_mode_fields(n, kbar, 0.1 * kbar, s), kbar,
                            gaussian_source(n, 2, c, 0.05), restart=30, tol=1e-8,
                            meta={"seed": seed0 + i}))
    return out


def config5_instance(seed: int, n: int = 255) -> Instance:
    """Learned-form workload: 255², k̄~U[10,30], σ=0.15k̄, s=4, degree 3 (Q=35),
    Gaussian (width 0.05) at a uniform point of [0.2,0.8]²."""
    rng = np.random.default_rng(seed)
    kbar = float(rng.uniform(10.0, 30.0))
    c = rng.uniform(0.2, 0.8, size=2)
    return Instance("c5_%05d" % seed, 2, n, 4, 3, sine_mode_fields(n, kbar, 0.15 * kbar, 4), kbar,
                    gaussian_source(n, 2, c, 0.05), restart=50, tol=1e-8, meta={"seed": seed})


# ------------------------------------------------------ paper's experiments

def one_d_paper(kbar: float, theta: float = 0.1, degree: int = 3, bc: str = "absorbing") -> Instance:
    """Section 6 model problem: k(ξ) = (1+θξ)k̄ constant in space, point source at 1/2,
    q from the mesh-size rule with maxk = k̄."""
    q = grid_rule_q(kbar)
    n = q + 2 if bc == "absorbing" else q
    k = np.empty((2, n))
    k[0] = kbar
    k[1] = theta * kbar
    return Instance("paper1d_k%g_t%g" % (kbar, theta), 1, n, 1, degree, k, kbar,
                    point_source(n, 1, bc), bc=bc, restart=10 ** 9, tol=1e-12,
                    meta={"q": q, "theta": theta})


def wedge_instance(degree: int, theta: float = 0.1, q: int = 127,
                   k123=(30.0, 15.0, 20.0)) -> Instance:
    """Section 7 wedge problem: k = (1+θξ_ℓ)k_ℓ on three regions split by the lines
    y = 0.2+0.1x and y = 0.6-0.2x (eq. stochastic_wavenumber_k123), point source at
    (1/2,1/2).  The mean k̄(x) is piecewise constant."""
    n = q + 2
    X, Y = _coords(n, 2)
    r1 = Y <= 0.2 + 0.1 * X
    r3 = 0.6 - 0.2 * X <= Y
    r2 = ~r1 & ~r3
    k = np.zeros((4, n * n))
    for l, (reg, kl) in enumerate(zip((r1, r2, r3), k123), start=1):
        k[0][reg] = kl
        k[l][reg] = theta * kl
    return Instance("wedge_r%d_t%g" % (degree, theta), 2, n, 3, degree, k, float("nan"),
                    point_source(n, 2), restart=10 ** 9, tol=1e-8, meta={"q": q, "theta": theta})
