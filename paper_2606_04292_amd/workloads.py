"""Seeded synthetic workloads for the NGS-FAS Richards solver.

This module only *describes* problems: grid shapes, boundary types, soil
parameters, initial states, and the seeded random inputs (a lognormal
saturated-conductivity field and a request stream).  It contains none of the
solver's arithmetic: no constitutive law, operator, sweep or transfer is
evaluated here.  Both the HIP library binding and the CPU oracle consume these
descriptions, each marshalling them into its own structures.

Conventions (paper section 2, with the vertex-centred reading of the grid):
  * ``dim`` in {1, 2, 3}; axis ``dim-1`` is the vertical axis and the vertical
    coordinate is elevation (bottom at 0, positive up).
  * ``n[l]`` nodes per axis including both boundary nodes, ``n = 2**k + 1``;
    node spacing ``h = L / (n - 1)``.
  * arrays are flattened with axis 0 fastest (the lexicographic flattening of
    section 2), i.e. numpy shape ``(n[dim-1], ..., n[0])`` in C order.
  * faces are numbered axis by axis: face ``2*l`` is the low end of axis ``l``
    and ``2*l+1`` its high end (so in any dimension the last two faces are
    bottom and top).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# Boundary-face kinds (shared numeric values of the C ABI and the oracle).
BC_DIRICHLET = 1
BC_NOFLUX = 2
BC_FREEDRAIN = 3
BC_DIRICHLET_STATE = 4  # prescribed head taken from the state (non-uniform boundary data)

# Constitutive models.
MODEL_VGM = 1         # van Genuchten - Mualem (l = 0.5)
MODEL_HAVERKAMP = 2   # Haverkamp et al.
MODEL_LINEAR = 3      # test-only law: theta affine in psi, K constant
MODEL_GARDNER = 4     # Gardner: theta and K exponential in psi

SINK_NONE = 0
SINK_FEDDES_EXP = 1   # Feddes-type a(psi) times an exponential root density

KAPPA_CONST = 1       # kappa_i = kappa
KAPPA_REL = 2         # kappa_i = kappa * m_ii
KAPPA_REMARK = 3      # kappa_i = max row sum of U minus row sum of U (Remark after the theorem)
COARSE_INJECT = 0     # coarse K* = fine K* at the coinciding node
COARSE_FW = 1         # coarse K* = full-weighting average of the finer level's K*

SEED_ROOT = 260604292


@dataclasses.dataclass
class GridSpec:
    dim: int
    n: List[int]                      # nodes per axis, length dim
    L: List[float]                    # extents (m), length dim
    face_bc: List[int]                # length 2*dim
    face_value: List[float]           # length 2*dim (used by Dirichlet faces)
    patch_face: int = -1              # one optional Dirichlet patch on a face
    patch_lo: Sequence[int] = (0, 0)  # tangential node-index range (inclusive)
    patch_hi: Sequence[int] = (0, 0)
    patch_value: float = 0.0

    @property
    def shape(self):
        """numpy shape (vertical axis first, axis 0 last)."""
        return tuple(reversed(self.n))

    @property
    def nodes(self) -> int:
        return int(np.prod(self.n))

    def levels(self) -> int:
        """Number of levels when every axis is halved until the shortest has 3 nodes."""
        m = min(self.n)
        k = 0
        while m > 3:
            m = (m - 1) // 2 + 1
            k += 1
        return k + 1


@dataclasses.dataclass
class LawSpec:
    model: int
    theta_s: float
    theta_r: float
    Ks: float
    vg_alpha: float = 0.0
    vg_n: float = 0.0
    hk_alpha: float = 0.0
    hk_beta: float = 0.0
    hk_A: float = 0.0
    hk_gamma: float = 0.0
    psi_unit: float = 1.0             # psi is multiplied by this before the law (100: cm)
    lin_c: float = 0.0                # MODEL_LINEAR: theta = theta_r + lin_c * psi
    sink: int = SINK_NONE
    Tp: float = 0.0                   # potential transpiration (m/s)
    root_len: float = 0.2             # e-folding depth of root density (m)
    h1: float = -0.1
    h2: float = -0.25
    h3: float = -4.0
    h4: float = -80.0
    xi: float = 0.0
    kappa_rule: int = KAPPA_REL
    kappa: float = 0.1
    newton_iters: int = 3             # pointwise Newton steps at most
    lag_extrap: int = 0               # BDF2 lag: 0 psi^n, 1 2 psi^n - psi^{n-1}
    newton_tol: float = 1e-10         # ... ending after a Newton step <= newton_tol |psi|
    gd_alpha: float = 0.0             # MODEL_GARDNER exponent (per law unit of psi)
    coarse_k: int = 0                 # COARSE_INJECT or COARSE_FW: K* on the coarse levels


@dataclasses.dataclass
class Workload:
    name: str
    grid: GridSpec
    law: LawSpec
    psi0: np.ndarray                  # initial state, grid.shape, float64
    dt: float
    steps: int
    order: int                        # 1 = BDF1, 2 = BDF2 (first step BDF1)
    Ks_field: Optional[np.ndarray] = None
    nu1: int = 2
    nu2: int = 2
    nu_coarse: int = 32
    # layered media: per-node soil index into soils (uint8, grid.shape); each
    # soil supplies the law's model, theta_s, theta_r, Ks and model parameters,
    # law supplies everything else
    soils: Optional[List[LawSpec]] = None
    soil_id: Optional[np.ndarray] = None


def _coords(grid: GridSpec):
    """Node coordinates as numpy arrays broadcastable to grid.shape."""
    out = []
    for l in range(grid.dim):
        x = np.arange(grid.n[l], dtype=np.float64) * (grid.L[l] / (grid.n[l] - 1))
        sh = [1] * grid.dim
        sh[grid.dim - 1 - l] = grid.n[l]
        out.append(x.reshape(sh))
    return out


def elevation(grid: GridSpec) -> np.ndarray:
    """Elevation of every node (for building initial states only)."""
    return np.broadcast_to(_coords(grid)[grid.dim - 1], grid.shape).copy()


def seed_sequence(*spawn_path: int) -> np.random.SeedSequence:
    ss = np.random.SeedSequence(SEED_ROOT)
    for k in spawn_path:
        ss = ss.spawn(k + 1)[k]
    return ss


def lognormal_field(shape, L, mean_lnK, sigma, corr_len, seed_path=(0,)):
    """Lognormal field exp(Y) on a vertex grid, Y Gaussian with covariance
    sigma^2 exp(-r^2 / corr_len^2), by circulant embedding on a periodic grid of
    twice the size, cropped.  Returns float64 array of ``shape``."""
    rng = np.random.default_rng(seed_sequence(*seed_path))
    dims = len(shape)
    spacing = [L[dims - 1 - a] / (shape[a] - 1) for a in range(dims)]
    big = [2 * (s - 1) for s in shape]
    r2 = np.zeros(big)
    for a in range(dims):
        idx = np.arange(big[a])
        d = np.minimum(idx, big[a] - idx) * spacing[a]
        sh = [1] * dims
        sh[a] = big[a]
        r2 = r2 + (d ** 2).reshape(sh)
    cov = sigma ** 2 * np.exp(-r2 / corr_len ** 2)
    lam = np.real(np.fft.fftn(cov))
    lam = np.clip(lam, 0.0, None)
    noise = rng.standard_normal(big) + 1j * rng.standard_normal(big)
    y = np.fft.ifftn(np.sqrt(lam) * noise) * math.sqrt(np.prod(big))
    y = np.real(y)[tuple(slice(0, s) for s in shape)]
    return np.exp(mean_lnK + y)


# ---------------------------------------------------------------------------
# The five configurations (full size) and shrunken copies for parity tests.
# ---------------------------------------------------------------------------

def config1(n: int = 257) -> Workload:
    """1-D column, 1 m, vGM, infiltration; BDF1, dt 60 s, 50 steps, V(2,2),
    3 Newton steps per cell (newton_tol 0: no early stop)."""
    g = GridSpec(dim=1, n=[n], L=[1.0], face_bc=[BC_DIRICHLET, BC_DIRICHLET],
                 face_value=[-5.0, -0.1])
    law = LawSpec(model=MODEL_VGM, theta_s=0.40, theta_r=0.08, Ks=1e-5,
                  vg_alpha=3.0, vg_n=2.0, newton_iters=3, newton_tol=0.0)
    psi0 = np.full(g.shape, -5.0)
    return Workload("col1d_vgm_%d" % n, g, law, psi0, dt=60.0, steps=50, order=1)


def config2(n: int = 513, ks_field: bool = True) -> Workload:
    """2-D slice 1x1 m, vGM with lognormal Ks, infiltration strip on the middle
    20 % of the top, no-flux elsewhere, free drainage at the bottom; BDF2,
    dt 30 s, 100 steps."""
    lo = int(math.ceil(0.4 * (n - 1)))
    hi = int(math.floor(0.6 * (n - 1)))
    g = GridSpec(dim=2, n=[n, n], L=[1.0, 1.0],
                 face_bc=[BC_NOFLUX, BC_NOFLUX, BC_FREEDRAIN, BC_NOFLUX],
                 face_value=[0.0, 0.0, 0.0, 0.0],
                 patch_face=3, patch_lo=(lo, 0), patch_hi=(hi, 0), patch_value=0.0)
    law = LawSpec(model=MODEL_VGM, theta_s=0.43, theta_r=0.05, Ks=1e-5,
                  vg_alpha=3.6, vg_n=1.56)
    ks = None
    if ks_field:
        ks = lognormal_field(g.shape, g.L, math.log(1e-5), 1.0, 0.1, seed_path=(0,))
    psi0 = np.full(g.shape, -1.0)
    return Workload("slice2d_vgm_lnks_%d" % n, g, law, psi0, dt=30.0, steps=100,
                    order=2, Ks_field=ks)


def config3(n: int = 257) -> Workload:
    """3-D block 1 m^3, Haverkamp (psi in cm), drainage from a hydrostatic
    saturated start to a bottom head of -1 m, no-flux elsewhere; BDF2,
    dt 120 s, 20 steps.  The stabilisation xi = 1e-4 /(m s) is needed here:
    the saturated start violates theta' > 0, and with the conductivity lagged
    over a 120 s step the cells next to the bottom boundary are over-drained
    and run away (psi -> -1e12 m, K* -> 0) when xi = 0."""
    g = GridSpec(dim=3, n=[n, n, n], L=[1.0, 1.0, 1.0],
                 face_bc=[BC_NOFLUX, BC_NOFLUX, BC_NOFLUX, BC_NOFLUX, BC_DIRICHLET, BC_NOFLUX],
                 face_value=[0.0, 0.0, 0.0, 0.0, -1.0, 0.0])
    law = LawSpec(model=MODEL_HAVERKAMP, theta_s=0.287, theta_r=0.075, Ks=9.4e-5,
                  hk_alpha=1.611e6, hk_beta=3.96, hk_A=1.175e6, hk_gamma=4.74,
                  psi_unit=100.0, xi=1e-4)
    psi0 = 1.0 - elevation(g)
    return Workload("block3d_haverkamp_%d" % n, g, law, psi0, dt=120.0, steps=20, order=2)


def config4(nx: int = 257, nz: int = 129) -> Workload:
    """3-D root uptake in a closed 1x1x0.5 m box, vGM, Feddes a(psi) with an
    exponential root density normalised to 5 mm/day; BDF2, dt 300 s, 48 steps."""
    g = GridSpec(dim=3, n=[nx, nx, nz], L=[1.0, 1.0, 0.5],
                 face_bc=[BC_NOFLUX] * 6, face_value=[0.0] * 6)
    law = LawSpec(model=MODEL_VGM, theta_s=0.45, theta_r=0.067, Ks=1.2e-6,
                  vg_alpha=2.0, vg_n=1.41, sink=SINK_FEDDES_EXP,
                  Tp=5e-3 / 86400.0, root_len=0.2)
    psi0 = np.full(g.shape, -1.0)
    return Workload("rootbox3d_vgm_%dx%dx%d" % (nx, nx, nz), g, law, psi0, dt=300.0,
                    steps=48, order=2)


def celia_column(n: int = 2049) -> Workload:
    """The 1-D infiltration benchmark of section 4.1 (after Celia et al.):
    a 40 cm Haverkamp column in cm and s, psi0 = -61.5 cm, Dirichlet -20.7 cm on
    top and -61.5 cm at the bottom, no sink, xi = 0, Lambda_kappa = 0.1 I,
    tau = 0.1 s, BDF1, V(5,5), run to t = 360 s."""
    g = GridSpec(dim=1, n=[n], L=[40.0], face_bc=[BC_DIRICHLET, BC_DIRICHLET],
                 face_value=[-61.5, -20.7])
    law = LawSpec(model=MODEL_HAVERKAMP, theta_s=0.287, theta_r=0.075, Ks=0.00944,
                  hk_alpha=1.611e6, hk_beta=3.96, hk_A=1.175e6, hk_gamma=4.74, psi_unit=1.0,
                  xi=0.0, kappa_rule=KAPPA_CONST, kappa=0.1)
    return Workload("celia_column%d" % n, g, law, np.full(n, -61.5), dt=0.1, steps=3600,
                    order=1, nu1=5, nu2=5)


# Soils of the layered 1-D column of section 4.1: the Haverkamp soil of the
# Celia benchmark and the Gardner and van Genuchten-Mualem soils the paper
# matches to it (alpha_G, n*, alpha_VG* as printed there; Ks, theta_s and
# theta_r shared; psi in cm).
CELIA_GARDNER_ALPHA = 0.01877      # 1/cm
CELIA_VG_N = 3.349
CELIA_VG_ALPHA = 0.03165           # 1/cm


def celia_soils() -> List[LawSpec]:
    """[Gardner, Haverkamp, vGM] soils of the layered column (section 4.1)."""
    common = dict(theta_s=0.287, theta_r=0.075, Ks=0.00944, psi_unit=1.0, xi=0.0,
                  kappa_rule=KAPPA_CONST, kappa=0.1)
    return [LawSpec(model=MODEL_GARDNER, gd_alpha=CELIA_GARDNER_ALPHA, **common),
            LawSpec(model=MODEL_HAVERKAMP, hk_alpha=1.611e6, hk_beta=3.96, hk_A=1.175e6,
                    hk_gamma=4.74, **common),
            LawSpec(model=MODEL_VGM, vg_alpha=CELIA_VG_ALPHA, vg_n=CELIA_VG_N, **common)]


def celia_composite(n: int = 2049) -> Workload:
    """The layered column of section 4.1: the Celia set-up with the composite
    law, Gardner for 30 <= z < 40 cm, Haverkamp for 20 <= z < 30 cm and vGM
    elsewhere (the printed half-open zones; the top node z = 40 falls in the
    vGM zone)."""
    w = celia_column(n)
    z = elevation(w.grid)
    sid = np.where((z >= 30.0) & (z < 40.0), 0, np.where((z >= 20.0) & (z < 30.0), 1, 2))
    soils = celia_soils()
    return dataclasses.replace(w, name="celia_composite%d" % n, law=soils[1], soils=soils,
                               soil_id=sid.astype(np.uint8))


def two_layer_vg(n: int = 257, steps: int = 175) -> Workload:
    """The two-layer infiltration of section 4.2: (0,100)^2 cm, vGM soils above
    and below the interface zeta(x) = 100 (0.1 (1 - cos(pi x / 100)) + 0.45),
    psi0 = -z, psi = 0 on top and bottom, no flux on the sides,
    Lambda_kappa = 0.1 I, xi = 0, tau = 0.01, FMG(10, 10) starts.  Reading:
    the paper gives Ks in cm/h but shows the solution in days up to 1.75 days,
    so time is in days (Ks converted, tau = 0.01 day, 175 steps)."""
    g = GridSpec(dim=2, n=[n, n], L=[100.0, 100.0],
                 face_bc=[BC_NOFLUX, BC_NOFLUX, BC_DIRICHLET, BC_DIRICHLET],
                 face_value=[0.0, 0.0, 0.0, 0.0])
    common = dict(model=MODEL_VGM, psi_unit=1.0, xi=0.0, kappa_rule=KAPPA_CONST, kappa=0.1)
    upper = LawSpec(theta_s=0.50, theta_r=0.120, vg_alpha=0.025, vg_n=3.00, Ks=0.25 * 24.0, **common)
    lower = LawSpec(theta_s=0.46, theta_r=0.034, vg_alpha=0.016, vg_n=1.37, Ks=2.00 * 24.0, **common)
    x, z = _coords(g)
    zeta = 100.0 * (0.1 * (1.0 - np.cos(np.pi * x / 100.0)) + 0.45)
    sid = np.broadcast_to(np.where(z >= zeta, 0, 1), g.shape).astype(np.uint8)
    psi0 = -elevation(g)
    return Workload("two_layer_vg%d" % n, g, upper, psi0, dt=0.01, steps=steps, order=1,
                    nu1=10, nu2=10, soils=[upper, lower], soil_id=np.ascontiguousarray(sid))


def gardner_2d(n: int = 129, steps: int = 30) -> Workload:
    """The 2-D Gardner infiltration of section 4.2: (0,10)^2 m, theta_s 0.45,
    theta_r 0.15, alpha 0.164 /m, Ks 0.1 m/day, psi0 = -10 m; on top the
    non-uniform head (1/alpha) ln(e^(-10 alpha) + (1 - e^(-10 alpha)) sin(pi x/10)),
    -10 m on the other boundaries; tau = 0.1 day for 3 days (30 steps), N = 128.
    The top values enter through the initial state (a DIRICHLET_STATE face).
    Not given by the paper for this case (readings): kappa and xi as in its
    1-D case (Lambda_kappa = 0.1 I, xi = 0), BDF1, V(5,5)."""
    g = GridSpec(dim=2, n=[n, n], L=[10.0, 10.0],
                 face_bc=[BC_DIRICHLET, BC_DIRICHLET, BC_DIRICHLET, BC_DIRICHLET_STATE],
                 face_value=[-10.0, -10.0, -10.0, 0.0])
    alpha = 0.164
    law = LawSpec(model=MODEL_GARDNER, theta_s=0.45, theta_r=0.15, Ks=0.1, gd_alpha=alpha,
                  psi_unit=1.0, xi=0.0, kappa_rule=KAPPA_CONST, kappa=0.1)
    x, _ = _coords(g)
    e = math.exp(-10.0 * alpha)
    top = np.log(e + (1.0 - e) * np.sin(np.pi * x.ravel() / 10.0)) / alpha
    psi0 = np.full(g.shape, -10.0)
    psi0[-1, :] = top
    return Workload("gardner2d_%d" % n, g, law, psi0, dt=0.1, steps=steps, order=1, nu1=5, nu2=5)


def serving_requests(count: int = 4096, seed_path=(1,)) -> List[Workload]:
    """The request stream: half 1-D columns (65..2049 nodes), half 2-D slices
    (65^2..513^2), random vGM parameters and infiltration/drainage boundaries,
    10 BDF2 steps of 60 s each."""
    rng = np.random.default_rng(seed_sequence(*seed_path))
    out = []
    for r in range(count):
        is2d = rng.random() < 0.5
        if is2d:
            n = int(rng.choice([65, 129, 257, 513]))
        else:
            n = int(rng.choice([65, 129, 257, 513, 1025, 2049]))
        alpha = rng.uniform(1.0, 5.0)
        vn = rng.uniform(1.3, 2.5)
        ks = 10.0 ** rng.uniform(-7.0, -4.0)
        ts = rng.uniform(0.35, 0.50)
        tr = rng.uniform(0.02, 0.10)
        infil = rng.random() < 0.5
        top = rng.uniform(-0.3, 0.0)
        bot = rng.uniform(-2.0, -0.5)
        p0 = rng.uniform(-3.0, -0.5)
        if is2d:
            if infil:
                fb = [BC_NOFLUX, BC_NOFLUX, BC_FREEDRAIN, BC_DIRICHLET]
                fv = [0.0, 0.0, 0.0, top]
            else:
                fb = [BC_NOFLUX, BC_NOFLUX, BC_DIRICHLET, BC_NOFLUX]
                fv = [0.0, 0.0, bot, 0.0]
            g = GridSpec(dim=2, n=[n, n], L=[1.0, 1.0], face_bc=fb, face_value=fv)
        else:
            if infil:
                fb, fv = [BC_FREEDRAIN, BC_DIRICHLET], [0.0, top]
            else:
                fb, fv = [BC_DIRICHLET, BC_NOFLUX], [bot, 0.0]
            g = GridSpec(dim=1, n=[n], L=[1.0], face_bc=fb, face_value=fv)
        law = LawSpec(model=MODEL_VGM, theta_s=ts, theta_r=tr, Ks=ks,
                      vg_alpha=alpha, vg_n=vn)
        psi0 = np.full(g.shape, p0)
        out.append(Workload("req%04d" % r, g, law, psi0, dt=60.0, steps=10, order=2))
    return out


def poisson_arrivals(count: int, rate: float, seed_path=(2,)) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed_sequence(*seed_path))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def shrink(w: Workload, n: int) -> Workload:
    """Same physics on a coarser grid with ``n`` nodes on the longest axis
    (2**k+1).  Used for parity tests that the oracle finishes in seconds."""
    g = w.grid
    nmax = max(g.n)
    ratio = (nmax - 1) // (n - 1)
    newn = [(m - 1) // ratio + 1 for m in g.n]
    lo = tuple(int(math.ceil(v / ratio)) for v in g.patch_lo)
    hi = tuple(int(v // ratio) for v in g.patch_hi)
    g2 = dataclasses.replace(g, n=newn, patch_lo=lo, patch_hi=hi)
    sl = tuple(slice(None, None, ratio) for _ in g.shape)
    psi0 = np.ascontiguousarray(w.psi0[sl])
    ks = None if w.Ks_field is None else np.ascontiguousarray(w.Ks_field[sl])
    return dataclasses.replace(w, name=w.name + "_n%d" % n, grid=g2, psi0=psi0, Ks_field=ks)
