"""Seeded synthetic workloads: scheme parameters and initial conserved moments.

This module is shared by the GPU path and by the FP64 oracle. It holds none of
the method's arithmetic: it only builds parameter dictionaries and initial
fields (point values at finest-cell centres, generated once on the host with
numpy so that both sides receive identical bits).

Parameter dictionary keys:
  scheme   "D1Q2" | "D1Q3" | "D2Q9" | "D2Q4E" | "D3Q6"
  jmin, jmax, eps, mu_bar, lam (lattice velocity), eq_param (V or alpha),
  velocity (V_x, V_y, V_z) of the D3Q6 advection,
  s        relaxation rate of every moment (0 for conserved moments)
  domain   (lo, hi) of the box along each axis
  bc       boundary of each side x-, x+, y-, y+ (BC_KINDS codes; default all
           periodic); bc_eval 0 / 1: wall values taken on the leaf / on the
           reconstruction (section "Boundary conditions")
Initial fields ``m0`` have shape [nc][N_J^d] with nc = 1 (1D, D3Q6), 3 (rho,
q_x, q_y) or 4 (the Euler system: rho, rho u, rho v, E), cell index x + N_J * y
(3D: x + N_J * (y + N_J * z)).
"""
from __future__ import annotations

import numpy as np

SCHEME_DIMS = {"D1Q2": (1, 2, 1), "D1Q3": (1, 3, 1), "D2Q9": (2, 9, 3), "D2Q4E": (2, 16, 4),
               "D3Q6": (3, 6, 1)}  # dim, q, conserved


BC_KINDS = {"periodic": 0, "copy": 1, "bounce_back": 2, "anti_bounce_back": 3}


def params(scheme: str, jmin: int, jmax: int, eps: float, s, mu_bar: float = 0.0, lam: float = 1.0,
           eq_param: float = 0.0, domain=(0.0, 1.0), bc=None, bc_eval: int = 0, gamma: int = 1,
           metric: str = "linf", velocity=(0.0, 0.0, 0.0)) -> dict:
    """Parameter dictionary. ``bc``: None (periodic) or the kind of each side
    x-, x+, y-, y+ (names of BC_KINDS or their codes; 1D takes two). ``gamma``:
    prediction stencil half-width 1..3; ``metric``: "linf" or "l2" sibling metric;
    ``velocity``: the D3Q6 advection velocity."""
    dim, q, _ = SCHEME_DIMS[scheme]
    s = [float(v) for v in s]
    assert len(s) == q
    codes = [0, 0, 0, 0]
    if bc is not None:
        for k, v in enumerate(bc):
            codes[k] = BC_KINDS[v] if isinstance(v, str) else int(v)
    return dict(scheme=scheme, dim=dim, q=q, jmin=int(jmin), jmax=int(jmax), eps=float(eps),
                mu_bar=float(mu_bar), lam=float(lam), eq_param=float(eq_param), s=s,
                domain=tuple(domain), bc=tuple(codes), bc_eval=int(bc_eval), gamma=int(gamma), metric=metric,
                velocity=tuple(float(v) for v in velocity))


def cell_centres(jmax: int, domain=(0.0, 1.0)) -> np.ndarray:
    lo, hi = domain
    n = 1 << jmax
    return lo + (np.arange(n) + 0.5) * (hi - lo) / n


def d2q9_s(s1: float, s2: float) -> list:
    """Relaxation vector diag(0, 0, 0, s1, s1, s1, s1, s2, s2) of the D2Q9 scheme."""
    return [0.0, 0.0, 0.0, s1, s1, s1, s1, s2, s2]


def s2_from_reynolds(re: float, u0: float, length: float, jmax: int, lam: float = 1.0) -> float:
    """Shear relaxation rate giving kinematic viscosity u0*length/re on level jmax
    (acoustic scaling, dt = dx/lam, c_s^2 = lam^2/3)."""
    nu = u0 * length / re
    dt = (length / (1 << jmax)) / lam
    cs2 = lam * lam / 3.0
    return 1.0 / (0.5 + nu / (cs2 * dt))


# ---------------------------------------------------------------- 1D workloads

def advection_d1q2(jmin=2, jmax=10, eps=1e-4, s=1.9, mu_bar=0.0, velocity=1.0):
    """D1Q2 linear advection on the periodic box [-1, 1]: indicator of [-0.3, 0.3]
    plus the bump exp(-50 x^2)."""
    cfg = params("D1Q2", jmin, jmax, eps, [0.0, s], mu_bar=mu_bar, lam=1.0, eq_param=velocity,
                 domain=(-1.0, 1.0))
    x = cell_centres(jmax, cfg["domain"])
    u0 = (np.abs(x) <= 0.3).astype(np.float64) + np.exp(-50.0 * x * x)
    return cfg, u0[None, :].copy()


def burgers_d1q3(jmin=2, jmax=14, eps=1e-4, s=1.5, mu_bar=0.0, alpha=0.5, seed=0, nmodes=8):
    """D1Q3 inviscid Burgers on the periodic box [-1, 1]: 0.5 * a normalised sum of
    `nmodes` sines with seeded U(-1, 1) amplitudes."""
    cfg = params("D1Q3", jmin, jmax, eps, [0.0, s, s], mu_bar=mu_bar, lam=1.0, eq_param=alpha,
                 domain=(-1.0, 1.0))
    x = cell_centres(jmax, cfg["domain"])
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, nmodes)
    u = sum(a[n - 1] * np.sin(np.pi * n * x) for n in range(1, nmodes + 1))
    u0 = 0.5 * u / np.max(np.abs(u))
    return cfg, u0[None, :].copy()


# ---------------------------------------------------------------- 2D workloads

def shear_layer_d2q9(jmin=3, jmax=10, eps=1e-3, mu_bar=1.0, re=1e4, u0=0.1, s1=1.5, width=1.0 / 80,
                     pert=0.05, seed=0):
    """D2Q9 double shear layer on the periodic unit square: u_x = u0 tanh((y-1/4)/w) for
    y <= 1/2 and u0 tanh((3/4-y)/w) above; u_y = pert*u0*sin(2 pi (x + phi)), phi seeded."""
    s2 = s2_from_reynolds(re, u0, 1.0, jmax)
    cfg = params("D2Q9", jmin, jmax, eps, d2q9_s(s1, s2), mu_bar=mu_bar, lam=1.0, domain=(0.0, 1.0))
    cfg.update(re=float(re), u0=float(u0))
    xc = cell_centres(jmax)
    X, Y = np.meshgrid(xc, xc, indexing="xy")  # [y][x]
    phi = np.random.default_rng(seed).uniform(0.0, 1.0)
    ux = np.where(Y <= 0.5, u0 * np.tanh((Y - 0.25) / width), u0 * np.tanh((0.75 - Y) / width))
    uy = pert * u0 * np.sin(2.0 * np.pi * (X + phi))
    rho = np.ones_like(ux)
    m0 = np.stack([rho.ravel(), (rho * ux).ravel(), (rho * uy).ravel()])
    return cfg, np.ascontiguousarray(m0)


def shear_layer_batch(n=96, jmin=3, seed=0, jmax_choices=(7, 8, 9, 10), eps_choices=(1e-2, 1e-3, 1e-4),
                      re_range=(1e3, 3e4)):
    """Independent D2Q9 shear layers with per-instance Re ~ U[1e3, 3e4], J in {7..10},
    eps in {1e-2, 1e-3, 1e-4}; instance i uses seed `seed + i` for its draws."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed + i)
        re = float(rng.uniform(*re_range))
        jmax = int(rng.choice(jmax_choices))
        eps = float(rng.choice(eps_choices))
        out.append(shear_layer_d2q9(jmin=jmin, jmax=jmax, eps=eps, re=re, seed=seed + 1000 + i))
    return out


def euler_s(sq=(1.9, 1.75, 1.75, 1.75), sxy=(1.0, 1.0, 1.0, 1.0)) -> list:
    """Relaxation vector of the vectorial D2Q4 scheme: per variable i the rates
    (0, s_i^q, s_i^q, s_i^xy) of its moments."""
    out = []
    for i in range(4):
        out += [0.0, float(sq[i]), float(sq[i]), float(sxy[i])]
    return out


def riemann_d2q4e(jmin=2, jmax=8, eps=1e-3, mu_bar=0.0, lam=5.0, gamma_gas=1.4, seed=0, bc="copy", gamma=1,
                  metric="linf"):
    """Euler system on [0, 1]^2 with the vectorial D2Q4 scheme (lambda = 5,
    s^q = 1.9 for rho and 1.75 for the others, s^xy = 1) and copy walls: a
    two-dimensional Riemann problem whose four quadrant states (x and y below
    or above 1/2) are drawn from a seeded generator, rho in [0.5, 1.5], u and v
    in [-0.5, 0.5], p in [0.2, 1.5] (a synthetic stand-in for the paper's
    configurations, whose states it does not print). ``gamma`` and ``metric``:
    the prediction half-width and sibling metric of the multiresolution."""
    cfg = params("D2Q4E", jmin, jmax, eps, euler_s(), mu_bar=mu_bar, lam=lam, eq_param=gamma_gas,
                 domain=(0.0, 1.0), bc=(bc,) * 4, gamma=gamma, metric=metric)
    rng = np.random.default_rng(seed)
    st = [(rng.uniform(0.5, 1.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), rng.uniform(0.2, 1.5))
          for _ in range(4)]  # quadrants LL, LR, UL, UR
    cfg.update(quadrant_states=st, gamma_gas=float(gamma_gas))
    xc = cell_centres(jmax)
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    q = (X > 0.5).astype(int) + 2 * (Y > 0.5).astype(int)
    rho, u, v, p = (np.choose(q, [s[k] for s in st]) for k in range(4))
    E = p / (gamma_gas - 1.0) + 0.5 * rho * (u * u + v * v)
    m0 = np.stack([rho.ravel(), (rho * u).ravel(), (rho * v).ravel(), E.ravel()])
    return cfg, np.ascontiguousarray(m0)


def random_vortex_d2q9(jmin=3, jmax=8, eps=1e-3, mu_bar=1.0, u0=0.05, s1=1.5, s2=1.8, seed=0, kmax=4):
    """D2Q9 on the periodic unit square with a smooth solenoidal velocity u0 * curl(psi)/|.|_inf,
    psi = sum over kx, ky in 1..kmax of a_k sin(2 pi (kx x + ky y) + phi_k), a_k ~ N(0,1)/|k|^2."""
    cfg = params("D2Q9", jmin, jmax, eps, d2q9_s(s1, s2), mu_bar=mu_bar, lam=1.0, domain=(0.0, 1.0))
    rng = np.random.default_rng(seed)
    ks = [(kx, ky) for ky in range(1, kmax + 1) for kx in range(1, kmax + 1)]
    amp = np.array([rng.normal() / (kx * kx + ky * ky) for kx, ky in ks])
    phs = rng.uniform(0.0, 2.0 * np.pi, len(ks))
    cfg.update(modes=ks, amplitudes=amp.tolist(), phases=phs.tolist(), u0=float(u0))
    return cfg, vortex_moments(cfg, amp)


def vortex_mode_fields(cfg: dict):
    """Velocity of each mode of `random_vortex_d2q9` at unit amplitude, before the
    max-norm scaling: arrays gx, gy of shape [modes][N_J^2] (cell index x + N_J y)."""
    xc = cell_centres(cfg["jmax"])
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    gx, gy = [], []
    for (kx, ky), p in zip(cfg["modes"], cfg["phases"]):
        c = np.cos(2.0 * np.pi * (kx * X + ky * Y) + p) * 2.0 * np.pi
        gx.append((c * ky).ravel())      # d psi / dy
        gy.append((-c * kx).ravel())     # -d psi / dx
    return np.array(gx), np.array(gy)


def vortex_moments(cfg: dict, amplitudes) -> np.ndarray:
    """Initial moments (rho = 1, q = u) of the vortex workload for the given mode
    amplitudes: u = u0 * g / max(|g_x|_inf, |g_y|_inf), g = sum_k a_k g_k."""
    gx, gy = vortex_mode_fields(cfg)
    a = np.asarray(amplitudes, np.float64)
    ux, uy = a @ gx, a @ gy
    scale = cfg["u0"] / max(np.max(np.abs(ux)), np.max(np.abs(uy)))
    m0 = np.stack([np.ones_like(ux), ux * scale, uy * scale])
    return np.ascontiguousarray(m0)


def vortex_amplitude_gradient(cfg: dict, mbar) -> np.ndarray:
    """dJ/da_k of the 16 mode amplitudes of the vortex workload from dJ/dm0
    ([3][N_J^2]): the transpose of the input map a -> m0 of vortex_moments,
    u = u0 g / S with g = sum_k a_k g_k and S the max norm of g over both
    components, differentiated at the cell that attains it."""
    gx, gy = vortex_mode_fields(cfg)
    a = np.asarray(cfg["amplitudes"], np.float64)
    ux, uy = a @ gx, a @ gy
    comp, vals = (gx, ux) if np.max(np.abs(ux)) >= np.max(np.abs(uy)) else (gy, uy)
    j = int(np.argmax(np.abs(vals)))
    S = abs(vals[j])
    dS = np.sign(vals[j]) * comp[:, j]
    s = cfg["u0"] / S
    mb = np.asarray(mbar, np.float64).reshape(3, -1)
    return s * (gx @ mb[1] + gy @ mb[2]) - (s / S) * dS * float(mb[1] @ ux + mb[2] @ uy)


# ---------------------------------------------------------------- 3D workload

def d3q6_s(s1: float = 1.4, s2: float = 1.0) -> list:
    """Relaxation vector diag(0, s1, s1, s1, s2, s2) of the D3Q6 scheme."""
    return [0.0, s1, s1, s1, s2, s2]


def ball_d3q6(jmin=1, jmax=8, eps=1e-3, mu_bar=2.0, s1=1.4, s2=1.0, velocity=(0.3, 0.2, 0.1), radius=0.15,
              gamma=1, metric="linf"):
    """D3Q6 advection of the indicator of the ball of radius 0.15 centred at the
    origin (section "Three dimensional advection equation": lambda = 1, s1 =
    1.4, s2 = 1, jmin = 1, J = 8, mu_bar = 2, eps = 1e-3), on the periodic box
    [-1, 1]^3. The paper does not state the velocity V nor the domain: V =
    (0.3, 0.2, 0.1) (each component below lambda / 3, where the equilibrium
    populations stay non-negative) and the box [-1, 1]^3 are this workload's
    choice."""
    cfg = params("D3Q6", jmin, jmax, eps, d3q6_s(s1, s2), mu_bar=mu_bar, lam=1.0, domain=(-1.0, 1.0),
                 gamma=gamma, metric=metric, velocity=velocity)
    cfg.update(radius=float(radius))
    xc = cell_centres(jmax, cfg["domain"])
    Z, Y, X = np.meshgrid(xc, xc, xc, indexing="ij")  # [z][y][x]
    u0 = (X * X + Y * Y + Z * Z <= radius * radius).astype(np.float64)
    return cfg, u0.reshape(1, -1).copy()


def random_field(cfg: dict, seed: int, kind: str = "smooth") -> np.ndarray:
    """Generic seeded initial conserved moments for tests: smooth random modes plus,
    for kind="jump", a step, so that meshes get several levels."""
    dim, q, nc = SCHEME_DIMS[cfg["scheme"]]
    n = 1 << cfg["jmax"]
    rng = np.random.default_rng(seed)
    xc = (np.arange(n) + 0.5) / n
    if dim == 1:
        grids = (xc,)
    elif dim == 2:
        X, Y = np.meshgrid(xc, xc, indexing="xy")
        grids = (X, Y)
    else:
        Z, Y, X = np.meshgrid(xc, xc, xc, indexing="ij")  # [z][y][x]: cell index x + N (y + N z)
        grids = (X, Y, Z)
    fields = []
    for c in range(nc):
        f = np.zeros_like(grids[0])
        for _ in range(3):
            k = rng.integers(1, 4, size=dim)
            ph = rng.uniform(0, 2 * np.pi)
            arg = sum(int(k[i]) * grids[i] for i in range(dim)) * 2 * np.pi + ph
            f = f + rng.uniform(-1, 1) * np.sin(arg)
        if kind == "jump":
            f = f + (grids[0] > 0.5 + 0.1 * rng.uniform(-1, 1)) * rng.uniform(0.5, 1.0)
        fields.append(f)
    if cfg["scheme"] == "D2Q9":
        rho = 1.0 + 0.05 * fields[0]
        ux = 0.05 * fields[1]
        uy = 0.05 * fields[2]
        m0 = np.stack([rho.ravel(), (rho * ux).ravel(), (rho * uy).ravel()])
    elif cfg["scheme"] == "D1Q3":
        u = fields[0]
        m0 = (0.4 * u / np.max(np.abs(u)))[None, :]
    else:
        m0 = fields[0].reshape(1, -1)
    return np.ascontiguousarray(m0, dtype=np.float64)
