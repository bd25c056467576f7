"""Plain CPU float64 oracle of semi-Lagrangian geodesic shooting for
Metamorphosis / LDDMM (François, Gori, Glaunès, arXiv:2106.08817).

TEST INFRASTRUCTURE ONLY. This module is the correctness reference for the HIP
library. Only the test-suite, the smoke check and the benchmark's CPU-baseline
leg may import it; the product path never does. It shares no code with the HIP
path and imports nothing from it.

Everything is whole-array NumPy in float64, with no blocking, fusion or
reordering beyond what the definitions state. Inputs given as float32 are
upcast to float64 (the same values the GPU receives).

Discretisation (readings of the paper, fixed here once):

* grid points q with unit spacing, last axis contiguous; time step dt = 1/T;
* mu := rho (the paper obtains LDDMM with rho = mu -> 0), so the velocity is
  v = -K * (z grad I) with no rho factor, the image gains rho * z, and the
  regulariser is lambda * (||v0||_V^2 + rho ||z0||^2);
* gradients: clamped central differences D_a;
* K: separable Gaussian, taps exp(-k^2 / 2 sigma^2) normalised to sum 1,
  truncated at |k| <= floor(3 sigma), zero padding outside the grid;
* interpolation: clamped (replicate-border) bilinear / trilinear;
* the momentum update multiplies the interpolated z by (1 - dt div v) with
  div v taken at the arrival point;
* norms are plain sums over grid points;
* the gradient is the exact derivative of this discrete cost; at a foot that
  sits exactly on a grid line the derivative is one-sided (cell floor(c)),
  and zero when the foot is clamped at or beyond a border.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

F64 = np.float64


def _as64(a) -> np.ndarray:
    return np.asarray(a, dtype=F64)


# ---------------------------------------------------------------------------
# Operators
# ---------------------------------------------------------------------------

def gaussian_taps(sigma: float) -> np.ndarray:
    """Normalised 1-D Gaussian taps w[k + r], |k| <= r = floor(3 sigma).

    Methods, Eq. 3 and the text after it: K is a Gaussian blurring kernel.
    Reading: truncated at three standard deviations and normalised to sum 1.
    """
    sigma = F64(sigma)
    if not (sigma > 0):
        raise ValueError("sigma must be positive")
    r = int(np.floor(3.0 * sigma))
    k = np.arange(-r, r + 1, dtype=F64)
    w = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return w / w.sum()


def conv_axis(f: np.ndarray, w: np.ndarray, axis: int) -> np.ndarray:
    """(g_a f)[q] = sum_k w[k] f[q + k e_a], zero outside the grid.

    One separable pass of the RKHS kernel (Methods, Eq. 3: K * .); fields of V
    vanish on the boundary of the domain, hence the zero padding."""
    f = _as64(f)
    r = (len(w) - 1) // 2
    pad = [(0, 0)] * f.ndim
    pad[axis] = (r, r)
    fp = np.pad(f, pad)
    n = f.shape[axis]
    out = np.zeros_like(f)
    for j, wk in enumerate(w):  # j = k + r
        sl = [slice(None)] * f.ndim
        sl[axis] = slice(j, j + n)
        out += wk * fp[tuple(sl)]
    return out


def smooth(f: np.ndarray, w: np.ndarray) -> np.ndarray:
    """G f = g_0 g_1 ... g_{d-1} f: the separable Gaussian over every axis."""
    out = _as64(f)
    for a in range(out.ndim):
        out = conv_axis(out, w, a)
    return out


def _shift_index(n: int, s: int) -> np.ndarray:
    return np.clip(np.arange(n) + s, 0, n - 1)


def diff(f: np.ndarray, axis: int) -> np.ndarray:
    """(D_a f)[q] = (f[q + e_a] - f[q - e_a]) / 2 with the index clamped to
    the grid (the image gradient of Methods, Eq. 3 on the grid)."""
    f = _as64(f)
    n = f.shape[axis]
    return 0.5 * (np.take(f, _shift_index(n, +1), axis=axis)
                  - np.take(f, _shift_index(n, -1), axis=axis))


def diff_T(g: np.ndarray, axis: int) -> np.ndarray:
    """Transpose of ``diff``: every clamped read of ``diff`` becomes an add."""
    g = _as64(g)
    n = g.shape[axis]
    gm = np.moveaxis(g, axis, 0)
    out = np.zeros_like(gm)
    np.add.at(out, _shift_index(n, +1), 0.5 * gm)
    np.add.at(out, _shift_index(n, -1), -0.5 * gm)
    return np.moveaxis(out, 0, axis)


@dataclass
class Feet:
    """Clamped multilinear interpolation data for foot points y [d, *shape]."""

    cell: Tuple[np.ndarray, ...]   # i_a = min(floor(c_a), n_a - 2)
    frac: Tuple[np.ndarray, ...]   # f_a = c_a - i_a in [0, 1]
    live: Tuple[np.ndarray, ...]   # chi_a = 1 iff 0 < y_a < n_a - 1 (strict)


def feet(y: np.ndarray, shape: Sequence[int]) -> Feet:
    """Cell and fraction of each foot point, clamped to the grid (bilinear /
    trilinear re-interpolation, semi-Lagrangian section)."""
    cells, fracs, lives = [], [], []
    for a, n in enumerate(shape):
        ya = _as64(y[a])
        c = np.clip(ya, 0.0, n - 1.0)
        i = np.minimum(np.floor(c), n - 2).astype(np.int64)
        cells.append(i)
        fracs.append(c - i)
        lives.append(((ya > 0.0) & (ya < n - 1.0)).astype(F64))
    return Feet(tuple(cells), tuple(fracs), tuple(lives))


def _corners(d: int):
    return list(itertools.product((0, 1), repeat=d))


def _weight(ft: Feet, b: Sequence[int], skip: int = -1) -> np.ndarray:
    w = 1.0
    for a, ba in enumerate(b):
        if a == skip:
            continue
        w = w * (ft.frac[a] if ba else 1.0 - ft.frac[a])
    return w


def interp(F: np.ndarray, ft: Feet) -> np.ndarray:
    """I(F; y) = sum over cell corners b of prod_a weight_a(b_a) F[i + b]."""
    F = _as64(F)
    out = 0.0
    for b in _corners(F.ndim):
        idx = tuple(i + ba for i, ba in zip(ft.cell, b))
        out = out + _weight(ft, b) * F[idx]
    return out


def interp_grad(F: np.ndarray, ft: Feet) -> List[np.ndarray]:
    """d I(F; y) / d y_a: the derivative of the multilinear weights along a,
    times chi_a (zero where the coordinate is clamped)."""
    F = _as64(F)
    d = F.ndim
    out = []
    for a in range(d):
        acc = 0.0
        for b in _corners(d):
            idx = tuple(i + bb for i, bb in zip(ft.cell, b))
            sign = 1.0 if b[a] else -1.0
            acc = acc + sign * _weight(ft, b, skip=a) * F[idx]
        out.append(ft.live[a] * acc)
    return out


def interp_T(a: np.ndarray, ft: Feet, shape: Sequence[int]) -> np.ndarray:
    """Transpose of ``interp``: each value is scattered with its weights onto
    the corners of its cell."""
    a = _as64(a)
    out = np.zeros(tuple(shape), dtype=F64)
    for b in _corners(len(shape)):
        idx = tuple(i + ba for i, ba in zip(ft.cell, b))
        np.add.at(out, idx, _weight(ft, b) * a)
    return out


def grid_coords(shape: Sequence[int]) -> np.ndarray:
    return np.stack(np.meshgrid(*[np.arange(n, dtype=F64) for n in shape], indexing="ij"))


# ---------------------------------------------------------------------------
# One step of the scheme and the shooting loop
# ---------------------------------------------------------------------------

def momentum_field(I: np.ndarray, z: np.ndarray) -> List[np.ndarray]:
    """m_a = z D_a I (the argument of K in the velocity of Methods, Eq. 3)."""
    return [_as64(z) * diff(I, a) for a in range(np.ndim(I))]


def velocity(I: np.ndarray, z: np.ndarray, w: np.ndarray) -> List[np.ndarray]:
    """v = -K * (z grad I) (Methods, Eq. 3, first line, with mu = rho)."""
    return [-smooth(m, w) for m in momentum_field(I, z)]


def divergence(v: Sequence[np.ndarray]) -> np.ndarray:
    """div v = sum_a D_a v_a on the grid (semi-Lagrangian section: the
    continuity characteristics still need an approximation of div v)."""
    return sum(diff(va, a) for a, va in enumerate(v))


def step_given_v(I, z, v, rho: float, dt: float):
    """Advance (I, z) by one semi-Lagrangian step for a given velocity v.

    Semi-Lagrangian section: I_{t+dt} ~ I_t o (Id - dt v_t); along the image
    characteristic dI/dt = mu z (Eqs. 5-6), along the momentum characteristic
    dz/dt = -(div v) z (Eqs. 7-9). Readings: the residual is added before the
    transport, I' = [I + rho dt z] o y (same gather as z), and the momentum
    factor is (1 - dt div v) at the arrival point."""
    I = _as64(I)
    z = _as64(z)
    shape = I.shape
    q = grid_coords(shape)
    y = np.stack([q[a] - dt * _as64(v[a]) for a in range(len(shape))])
    ft = feet(y, shape)
    Ih = interp(I, ft)
    zh = interp(z, ft)
    delta = divergence(v)
    I1 = Ih + rho * dt * zh
    z1 = zh * (1.0 - dt * delta)
    return I1, z1, dict(y=y, feet=ft, Ihat=Ih, zhat=zh, delta=delta)


def step(I, z, rho: float, dt: float, w: np.ndarray):
    """One full step: velocity from (I, z), then the semi-Lagrangian update."""
    v = velocity(I, z, w)
    I1, z1, aux = step_given_v(I, z, v, rho, dt)
    aux["v"] = v
    return I1, z1, aux


def step_eulerian_given_v(I, z, v, rho: float, dt: float):
    """One step of the Eulerian scheme the paper compares against (option 1 of
    the semi-Lagrangian section; Eq. 5 and the continuity equation integrated
    at fixed grid points): explicit Euler in time with the same clamped central
    differences D as the rest of the scheme,
    I' = I - dt sum_a v_a D_a I + rho dt z,   z' = z - dt sum_a D_a (z v_a).
    Readings: the paper names the scheme but not its discretisation."""
    I = _as64(I)
    z = _as64(z)
    d = I.ndim
    adv = sum(_as64(v[a]) * diff(I, a) for a in range(d))
    flux = sum(diff(z * _as64(v[a]), a) for a in range(d))
    return I - dt * adv + rho * dt * z, z - dt * flux


def step_mixed_given_v(I, z, v, rho: float, dt: float):
    """Option 3 of the semi-Lagrangian section: the image is moved
    semi-Lagrangianly (as in step_given_v) and the momentum by the Eulerian
    continuity update of step_eulerian_given_v."""
    I1, _, _ = step_given_v(I, z, v, rho, dt)
    _, z1 = step_eulerian_given_v(I, z, v, rho, dt)
    return I1, z1


SCHEMES = ("sl", "eulerian", "mixed")


@dataclass
class Trajectory:
    I: List[np.ndarray]          # I_0 .. I_T
    z: List[np.ndarray]          # z_0 .. z_T
    v: List[List[np.ndarray]]    # v_0 .. v_{T-1}


def shoot(S, p0, rho: float, sigma: float, T: int, scheme: str = "sl") -> Trajectory:
    """Geodesic shooting from (I_0, z_0) = (S, p0) over T steps of dt = 1/T
    (Methods, Eq. 3 integrated with the full semi-Lagrangian scheme; scheme
    "eulerian" or "mixed" integrates with the alternatives the paper compares,
    step_eulerian_given_v and step_mixed_given_v, from the same velocity)."""
    if T < 1:
        raise ValueError("T must be >= 1")
    if scheme not in SCHEMES:
        raise ValueError(f"scheme must be one of {SCHEMES}")
    w = gaussian_taps(sigma)
    dt = 1.0 / T
    I, z = _as64(S).copy(), _as64(p0).copy()
    Is, zs, vs = [I], [z], []
    for _ in range(T):
        if scheme == "sl":
            I, z, aux = step(I, z, F64(rho), dt, w)
            v = aux["v"]
        else:
            v = velocity(I, z, w)
            fn = step_eulerian_given_v if scheme == "eulerian" else step_mixed_given_v
            I, z = fn(I, z, v, F64(rho), dt)
        vs.append(v)
        Is.append(I)
        zs.append(z)
    return Trajectory(Is, zs, vs)


def deformation(S, p0, rho: float, sigma: float, T: int, traj: Trajectory = None) -> np.ndarray:
    """Deformation map of the shot, psi_T (the deformation grids of the Results
    section, obtained by integrating over every v_t; the flow of Methods,
    d phi / dt = v o phi, discretised semi-Lagrangianly): psi_0 = Id and
    psi_{t+1} = psi_t o (Id - dt v_t), i.e. every component of psi_t is
    re-interpolated at the feet of step t with the clamped multilinear weights
    that move I and z. psi_T maps the arrival grid back into the source, so for
    rho = 0, I_T ~ S o psi_T. Returns [d, *shape] in grid coordinates
    (component a along array axis a)."""
    if traj is None:
        traj = shoot(S, p0, rho, sigma, T)
    shape = np.shape(S)
    d = len(shape)
    dt = 1.0 / T
    q = grid_coords(shape)
    psi = q.copy()
    for t in range(T):
        v = traj.v[t]
        ft = feet(np.stack([q[a] - dt * _as64(v[a]) for a in range(d)]), shape)
        psi = np.stack([interp(psi[a], ft) for a in range(d)])
    return psi


def cost_terms(S, J, p0, rho: float, sigma: float, lam: float, T: int, traj: Trajectory = None):
    """(H, data, reg) of the inexact matching cost (Methods, Eq. 4):
    H = 1/2 ||I_1 - J||^2 + lambda (||v0||_V^2 + rho ||z0||^2) with
    ||v0||_V^2 = <z0 grad S, K * (z0 grad S)>."""
    if traj is None:
        traj = shoot(S, p0, rho, sigma, T)
    w = gaussian_taps(sigma)
    data = 0.5 * np.sum((traj.I[-1] - _as64(J)) ** 2)
    m0 = momentum_field(S, p0)
    normV = sum(np.sum(m * smooth(m, w)) for m in m0)
    reg = normV + F64(rho) * np.sum(_as64(p0) ** 2)
    return data + F64(lam) * reg, data, F64(lam) * reg


def cost(S, J, p0, rho, sigma, lam, T) -> float:
    return cost_terms(S, J, p0, rho, sigma, lam, T)[0]


# ---------------------------------------------------------------------------
# Hand-written discrete adjoint (exact gradient of the discrete cost)
# ---------------------------------------------------------------------------

def step_adjoint(I, z, v, Ibar1, zbar1, rho: float, dt: float, w: np.ndarray, extra_mbar=None):
    """Reverse one step: given the cotangents (Ibar_{t+1}, zbar_{t+1}) of the
    step output, return (Ibar_t, zbar_t) for its input (I_t, z_t), where the
    step is ``step`` with v = -G(z grad I) and G built from the taps ``w``.
    ``extra_mbar`` is added to the cotangent of m = z grad I (the
    regulariser's contribution at t = 0)."""
    I = _as64(I)
    z = _as64(z)
    Ibar1 = _as64(Ibar1)
    zbar1 = _as64(zbar1)
    d = I.ndim
    shape = I.shape
    q = grid_coords(shape)
    y = np.stack([q[a] - dt * _as64(v[a]) for a in range(d)])
    ft = feet(y, shape)
    zh = interp(z, ft)
    delta = divergence(v)
    # I' = Ih + rho dt zh ;  z' = zh (1 - dt delta)
    zh_bar = rho * dt * Ibar1 + (1.0 - dt * delta) * zbar1
    delta_bar = -dt * zh * zbar1
    Ibar = interp_T(Ibar1, ft, shape)
    zbar = interp_T(zh_bar, ft, shape)
    gI = interp_grad(I, ft)
    gz = interp_grad(z, ft)
    # y_a = q_a - dt v_a, delta = sum_a D_a v_a
    vbar = [-dt * (Ibar1 * gI[a] + zh_bar * gz[a]) + diff_T(delta_bar, a) for a in range(d)]
    # v_a = -G m_a with G symmetric (zero-padded symmetric taps)
    mbar = [-smooth(vb, w) for vb in vbar]
    if extra_mbar is not None:
        mbar = [mb + _as64(e) for mb, e in zip(mbar, extra_mbar)]
    # m_a = z D_a I
    for a in range(d):
        zbar = zbar + mbar[a] * diff(I, a)
        Ibar = Ibar + diff_T(z * mbar[a], a)
    return Ibar, zbar


def cost_and_grad(S, J, p0, rho: float, sigma: float, lam: float, T: int):
    """Return (H, dH/dp0, dH/dS, (data, reg)) by the discrete adjoint of the
    whole shooting loop (the derivative that automatic differentiation of the
    discrete program gives, Results: autodiff replaces deriving the adjoint).
    The trajectory is stored in full."""
    rho = F64(rho)
    lam = F64(lam)
    w = gaussian_taps(sigma)
    dt = 1.0 / T
    traj = shoot(S, p0, rho, sigma, T)
    H, data, reg = cost_terms(S, J, p0, rho, sigma, lam, T, traj)
    Ibar = traj.I[-1] - _as64(J)
    zbar = np.zeros_like(Ibar)
    for t in range(T - 1, -1, -1):
        extra = None
        if t == 0:
            # d/dm0 of lam * <m0, G m0> = 2 lam G m0 = -2 lam v0
            extra = [-2.0 * lam * va for va in traj.v[0]]
        Ibar, zbar = step_adjoint(traj.I[t], traj.z[t], traj.v[t], Ibar, zbar,
                                     rho, dt, w, extra)
    grad_p0 = zbar + 2.0 * lam * rho * _as64(p0)
    return H, grad_p0, Ibar, (data, reg)


def max_displacement(traj: Trajectory, T: int) -> float:
    """max over steps, points and axes of |dt v| (pixels moved per step)."""
    dt = 1.0 / T
    return max(float(np.abs(dt * va).max()) for vt in traj.v for va in vt)


def energy(I, z, rho: float, w: np.ndarray) -> float:
    """||v||_V^2 + rho ||z||^2 at one time (conserved by the continuous
    geodesic: Methods, remark after Eq. 3). Diagnostic only."""
    m = momentum_field(I, z)
    return float(sum(np.sum(mm * smooth(mm, w)) for mm in m) + rho * np.sum(_as64(z) ** 2))


def gradient_descent(S, J, p0, rho, sigma, lam, T, iters: int, eta: float = 1.0):
    """Fixed-step gradient descent on p0 (Results: all costs are optimised by
    gradient descent); the step is halved whenever the cost rises."""
    p = _as64(p0).copy()
    H_prev = None
    history = []
    for _ in range(iters):
        H, g, _, _ = cost_and_grad(S, J, p, rho, sigma, lam, T)
        if H_prev is not None and H > H_prev:
            eta *= 0.5
        history.append(H)
        H_prev = H
        p = p - eta * g
    return p, history
