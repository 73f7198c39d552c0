"""Seeded synthetic initial states for the rotating shallow-water model.

Every function here builds *inputs* from continuous closed forms evaluated at
cell centres (spherical harmonics, zonal profiles, Gaussian bumps) -- none of
the finite-volume operators or integrator arithmetic appears here.

State layout (Sec. 2, eq. dynu): u = (u_x | u_y | u_z | h), each block N long,
velocity in Cartesian components tangent to the sphere, h in metres.
"""
import numpy as np

from .rng import Stream, BASE_SEED
from .mesh import get_mesh

RADIUS = 6.371e6
OMEGA = 7.292e-5
GRAVITY = 9.80616


# --------------------------------------------------------------------------
# real orthonormal spherical harmonics
# --------------------------------------------------------------------------
def _legendre_table(mu, cth, lmax):
    """Fully normalised associated Legendre functions Pbar[l][m](mu), l<=lmax."""
    P = [[None] * (lmax + 1) for _ in range(lmax + 1)]
    P[0][0] = np.full_like(mu, np.sqrt(1.0 / (4.0 * np.pi)))
    for m in range(1, lmax + 1):
        P[m][m] = -np.sqrt((2.0 * m + 1.0) / (2.0 * m)) * cth * P[m - 1][m - 1]
    for m in range(0, lmax):
        P[m + 1][m] = np.sqrt(2.0 * m + 3.0) * mu * P[m][m]
    for m in range(0, lmax + 1):
        for l in range(m + 2, lmax + 1):
            a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            P[l][m] = a * (mu * P[l - 1][m] - b * P[l - 2][m])
    return P


def sh_eval(coef, xyz, lmax):
    """sum_{l,m} coef[(l,m)] Y_lm(x) for unit vectors x (real, orthonormal).

    coef is a dict (l, m) -> value, m in [-l, l]; m<0 are the sine terms.
    """
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    mu = np.clip(z, -1.0, 1.0)
    cth = np.sqrt(np.maximum(0.0, x * x + y * y))
    lon = np.arctan2(y, x)
    P = _legendre_table(mu, cth, lmax)
    out = np.zeros_like(mu)
    for (l, m), c in coef.items():
        if m == 0:
            out += c * P[l][0]
        elif m > 0:
            out += c * np.sqrt(2.0) * P[l][m] * np.cos(m * lon)
        else:
            out += c * np.sqrt(2.0) * P[l][-m] * np.sin(-m * lon)
    return out


def _tangent_basis(xyz):
    ref = np.where(np.abs(xyz[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]),
                   np.array([[1.0, 0.0, 0.0]]))
    e1 = np.cross(ref, xyz)
    e1 /= np.linalg.norm(e1, axis=1)[:, None]
    e2 = np.cross(xyz, e1)
    return e1, e2


def surface_gradient(fun, xyz, radius=RADIUS, delta=1e-5):
    """Gradient on the sphere of a smooth function given as a callable of unit
    vectors, by central differences along two tangent great circles."""
    e1, e2 = _tangent_basis(xyz)
    ang = np.arctan(delta)
    g = np.zeros_like(xyz)
    for e in (e1, e2):
        xp = xyz + delta * e
        xm = xyz - delta * e
        xp /= np.linalg.norm(xp, axis=1)[:, None]
        xm /= np.linalg.norm(xm, axis=1)[:, None]
        d = (fun(xp) - fun(xm)) / (2.0 * ang * radius)
        g += d[:, None] * e
    return g


def random_sh_coef(stream, lmin=1, lmax=16):
    """c_lm ~ N(0, sigma_l^2), sigma_l^2 = l^-2/(2l+1): degree power ~ l^-2."""
    coef = {}
    for l in range(lmin, lmax + 1):
        z = stream.normal(2 * l + 1)
        s = np.sqrt(l ** -2.0 / (2 * l + 1))
        for k, m in enumerate(range(-l, l + 1)):
            coef[(l, m)] = s * z[k]
    return coef


def sh_perturbation(stream, xyz, amplitude, lmax=16):
    """Seeded SH field (degrees 1..lmax) scaled to max|h'| = amplitude.

    Returns (h', callable) where the callable evaluates the same scaled
    continuous field at arbitrary unit vectors."""
    coef = random_sh_coef(stream, 1, lmax)
    raw = sh_eval(coef, xyz, lmax)
    scale = amplitude / np.max(np.abs(raw))
    fun = lambda p: scale * sh_eval(coef, p, lmax)
    return scale * raw, fun


def balanced_velocity(fun, xyz, g=GRAVITY, omega=OMEGA, radius=RADIUS):
    """u = g/(2 Omega) * sin(lat)/(sin^2(lat) + sin^2(10 deg)) * (n x grad h').

    Geostrophic away from the equator, tapered to zero at it (f = 0 there)."""
    grad = surface_gradient(fun, xyz, radius)
    s = xyz[:, 2]
    taper = s / (s * s + np.sin(np.deg2rad(10.0)) ** 2)
    return (g / (2.0 * omega)) * taper[:, None] * np.cross(xyz, grad)


def zonal_unit(xyz):
    """Unit eastward vector e_phi at each point (zero at the poles)."""
    e = np.stack([-xyz[:, 1], xyz[:, 0], np.zeros(len(xyz))], 1)
    n = np.linalg.norm(e, axis=1)
    return e / np.where(n > 0, n, 1.0)[:, None]


def solid_body(xyz, u0, h_eq, g=GRAVITY, omega=OMEGA, radius=RADIUS):
    """Zonal solid-body flow u = u0 cos(lat) and its balanced depth
    (closed-form integral of g dh/dlat = -a u (f + u tan(lat)/a))."""
    s = xyz[:, 2]
    c = np.sqrt(np.maximum(0.0, 1.0 - s * s))
    vel = (u0 * c)[:, None] * zonal_unit(xyz)
    h = h_eq - (radius * omega * u0 + 0.5 * u0 * u0) * s * s / g
    return vel, h


def jet_profile(lat, umax=80.0, lat0=np.deg2rad(45.0), half=np.deg2rad(25.0)):
    xi = (lat - lat0) / half
    out = np.zeros_like(lat)
    inside = np.abs(xi) < 1.0
    out[inside] = umax * np.exp(1.0 - 1.0 / (1.0 - xi[inside] ** 2))
    return out


def zonal_jet(xyz, h_mean, g=GRAVITY, omega=OMEGA, radius=RADIUS, npts=400001):
    """Narrow balanced jet (C-infinity bump in latitude between 20N and 70N)
    with depth from the gradient-wind balance, integrated numerically and
    shifted to the given area-mean depth."""
    from scipy.integrate import cumulative_trapezoid
    lat_g = np.linspace(-np.pi / 2, np.pi / 2, npts)
    u = jet_profile(lat_g)
    f = 2.0 * omega * np.sin(lat_g)
    rhs = -(radius * u * f + u * u * np.tan(np.clip(lat_g, -1.5707963, 1.5707963))) / g
    rhs[0] = rhs[-1] = 0.0
    hg = cumulative_trapezoid(rhs, lat_g, initial=0.0)
    mean = np.trapezoid(hg * np.cos(lat_g), lat_g) / 2.0
    hg += h_mean - mean
    lat = np.arcsin(np.clip(xyz[:, 2], -1.0, 1.0))
    h = np.interp(lat, lat_g, hg)
    vel = jet_profile(lat)[:, None] * zonal_unit(xyz)
    return vel, h


def gaussian_bump(xyz, centre, amp=120.0, r=1.0 / 3.0):
    d = np.arccos(np.clip(xyz @ centre, -1.0, 1.0))
    return amp * np.exp(-(d / r) ** 2)


def random_point(stream, lat_lo=-np.pi / 2, lat_hi=np.pi / 2):
    """Uniform on the sphere restricted to a latitude band."""
    u = stream.uniform(2)
    z = np.sin(lat_lo) + (np.sin(lat_hi) - np.sin(lat_lo)) * u[0]
    lon = 2.0 * np.pi * u[1]
    c = np.sqrt(1.0 - z * z)
    return np.array([c * np.cos(lon), c * np.sin(lon), z])


def pack(vel, h):
    return np.ascontiguousarray(np.concatenate([vel[:, 0], vel[:, 1], vel[:, 2], h]))


# --------------------------------------------------------------------------
# workload recipes
# --------------------------------------------------------------------------
def sh_balanced_state(level, seed, amplitude=100.0, depth=5000.0, stream_id=1):
    """h = depth + SH(amplitude) (degrees 1-16, spectrum ~ l^-2), u balanced."""
    m = get_mesh(level)
    xyz = m["xyz"]
    hp, fun = sh_perturbation(Stream(seed, stream_id), xyz, amplitude)
    vel = balanced_velocity(fun, xyz)
    return pack(vel, depth + hp)


def solid_body_bump_state(level, seed, u0=38.6, h_eq=5000.0):
    m = get_mesh(level)
    xyz = m["xyz"]
    vel, h = solid_body(xyz, u0, h_eq)
    c = random_point(Stream(seed, 2))
    return pack(vel, h + gaussian_bump(xyz, c))


def mountain(level, seed, height=1500.0, r=0.3):
    """Synthetic terrain h_s: one smooth Gaussian mountain (height in metres,
    angular radius r) at a seeded point between 20 and 60 degrees north."""
    m = get_mesh(level)
    c = random_point(Stream(seed, 7), np.deg2rad(20.0), np.deg2rad(60.0))
    return gaussian_bump(m["xyz"], c, amp=height, r=r)


def mountain_flow_state(level, seed, u0=20.0, h_eq=5000.0, height=1500.0):
    """Solid-body zonal flow over the seeded mountain: the free surface
    h + h_s is the balanced solid-body surface, so the depth is h = that
    surface minus h_s (the flow is unbalanced only through the mountain)."""
    m = get_mesh(level)
    vel, h = solid_body(m["xyz"], u0, h_eq)
    return pack(vel, h - mountain(level, seed, height))


def jet_bump_state(level, seed, h_mean=10000.0):
    m = get_mesh(level)
    xyz = m["xyz"]
    vel, h = zonal_jet(xyz, h_mean)
    c = random_point(Stream(seed, 3), np.deg2rad(20.0), np.deg2rad(70.0))
    return pack(vel, h + gaussian_bump(xyz, c))


def ensemble_states(level, seed, members=64):
    """Member k: h = 5000 + SH(a_k), a_k ~ U[10, 200] m, balanced u;
    step sizes drawn uniformly from {600, 1200, 2400, 3600} s."""
    st = Stream(seed, 4)
    amps = 10.0 + 190.0 * st.uniform(members)
    dts = np.array([600.0, 1200.0, 2400.0, 3600.0])[st.integers(members, 4)]
    m = get_mesh(level)
    xyz = m["xyz"]
    U = np.empty((members, 4 * len(xyz)))
    for k in range(members):
        hp, fun = sh_perturbation(Stream(seed, 100 + k), xyz, amps[k])
        U[k] = pack(balanced_velocity(fun, xyz), 5000.0 + hp)
    return U, dts


def adjoint_twin(level, seed, steps=12, n_obs=5000, truth_amp=20.0, noise=5.0):
    """Inputs of the twin experiment of the adjoint workload: the initial
    state (as sh_balanced_state), the truth's initial state (that state plus
    an independent SH(truth_amp) depth perturbation with its balanced
    velocity), n_obs distinct (step, cell) pairs with step in 1..steps, drawn
    uniformly without replacement, and N(0, noise^2) observation errors.
    The observations are y = h_truth(step, cell) + error, with h_truth from
    the caller's own integration of the truth."""
    xyz = get_mesh(level)["xyz"]
    n = len(xyz)
    u0 = sh_balanced_state(level, seed)
    hp, fun = sh_perturbation(Stream(seed, 7), xyz, truth_amp)
    ut = u0 + pack(balanced_velocity(fun, xyz), hp)
    st = Stream(seed, 8)
    total = steps * n
    if n_obs > total:
        raise ValueError("more observations than (step, cell) pairs")
    chosen, seen = [], set()
    while len(chosen) < n_obs:
        for k in st.integers(2 * (n_obs - len(chosen)), total):
            k = int(k)
            if k not in seen:
                seen.add(k)
                chosen.append(k)
                if len(chosen) == n_obs:
                    break
    idx = np.array(chosen, dtype=np.int64)
    return u0, ut, 1 + idx // n, idx % n, noise * st.normal(n_obs)


def config_seed(index):
    return BASE_SEED + index


# Physical/model parameters of each workload (gamma_h per the readings:
# 4e-4 by default, 1.25e-2 for the jet).
WORKLOADS = {
    "c1_exprb42_l4": dict(level=4, gamma_h=4e-4, tol=1e-10, m_max=40),
    "c2_l6_24x3600": dict(level=6, gamma_h=4e-4, tol=1e-10, m_max=40),
    "c3_l8_jet": dict(level=8, gamma_h=1.25e-2, tol=1e-10, m_max=40),
    "c4_l6_ensemble64": dict(level=6, gamma_h=4e-4, tol=1e-10, m_max=40),
    "c5_l7_adjoint": dict(level=7, gamma_h=4e-4, tol=1e-10, m_max=40),
}


def initial_state(name, level=None):
    """Initial state of a named workload (optionally on another grid level,
    same recipe) -- used for the small parity cases."""
    idx = {"c1": 0, "c2": 1, "c3": 2, "c4": 3, "c5": 4}[name[:2]]
    seed = config_seed(idx)
    lev = WORKLOADS[name]["level"] if level is None else level
    if idx in (0, 4):
        return sh_balanced_state(lev, seed)
    if idx == 1:
        return solid_body_bump_state(lev, seed)
    if idx == 2:
        return jet_bump_state(lev, seed)
    U, _ = ensemble_states(lev, seed, 1)
    return U[0]
