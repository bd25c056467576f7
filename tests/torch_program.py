"""An independent float64 torch program of the same discrete scheme and cost,
differentiated by torch autograd. Test infrastructure: it pins the oracle's
hand-written adjoint (tests only; written without the oracle's code).

Readings shared with the oracle by definition (not by code): unit grid
spacing, dt = 1/T, clamped central differences, normalised Gaussian taps
truncated at floor(3 sigma) with zero padding, clamped multilinear
interpolation whose derivative vanishes at or beyond a border, foot cell
floor(c) (one-sided derivative on grid lines), mu = rho.
"""
import math

import torch

torch.set_default_dtype(torch.float64)


def taps(sigma):
    r = math.floor(3.0 * float(sigma))
    k = torch.arange(-r, r + 1, dtype=torch.float64)
    g = torch.exp(-0.5 * (k / float(sigma)) ** 2)
    return g / g.sum()


def blur_axis(f, w, axis):
    # move the axis last, flatten the others, zero-padded conv1d (w is symmetric)
    x = f.movedim(axis, -1)
    shp = x.shape
    x = x.reshape(-1, 1, shp[-1])
    r = (w.numel() - 1) // 2
    y = torch.nn.functional.conv1d(x, w.view(1, 1, -1), padding=r)
    return y.reshape(shp).movedim(-1, axis)


def blur(f, w):
    for a in range(f.dim()):
        f = blur_axis(f, w, a)
    return f


def grad_axis(f, axis):
    n = f.shape[axis]
    up = torch.cat([f.narrow(axis, 1, n - 1), f.narrow(axis, n - 1, 1)], dim=axis)
    dn = torch.cat([f.narrow(axis, 0, 1), f.narrow(axis, 0, n - 1)], dim=axis)
    return 0.5 * (up - dn)


def sample(F, y):
    """Clamped multilinear interpolation of F at coordinates y [d, *shape]."""
    d = F.dim()
    cells, fr = [], []
    for a in range(d):
        n = F.shape[a]
        inside = (y[a] > 0) & (y[a] < n - 1)
        c = torch.where(inside, y[a], y[a].detach().clamp(0, n - 1))
        i = torch.clamp(torch.floor(c.detach()), max=n - 2).long()
        cells.append(i)
        fr.append(c - i.to(c.dtype))
    out = 0.0
    for corner in range(2 ** d):
        bits = [(corner >> (d - 1 - a)) & 1 for a in range(d)]
        wgt = 1.0
        idx = []
        for a, b in enumerate(bits):
            wgt = wgt * (fr[a] if b else 1.0 - fr[a])
            idx.append(cells[a] + b)
        out = out + wgt * F[tuple(idx)]
    return out


def shoot(S, p0, rho, sigma, T):
    w = taps(sigma)
    dt = 1.0 / T
    d = S.dim()
    q = torch.stack(torch.meshgrid(*[torch.arange(n, dtype=torch.float64) for n in S.shape],
                                   indexing="ij"))
    I, z = S, p0
    vs = []
    for _ in range(T):
        v = [-blur(z * grad_axis(I, a), w) for a in range(d)]
        vs.append(v)
        y = torch.stack([q[a] - dt * v[a] for a in range(d)])
        Ih = sample(I, y)
        zh = sample(z, y)
        div = sum(grad_axis(v[a], a) for a in range(d))
        I, z = Ih + rho * dt * zh, zh * (1.0 - dt * div)
    return I, z, vs


def cost(S, J, p0, rho, sigma, lam, T):
    w = taps(sigma)
    I1, _, _ = shoot(S, p0, rho, sigma, T)
    m0 = [p0 * grad_axis(S, a) for a in range(S.dim())]
    normV = sum((m * blur(m, w)).sum() for m in m0)
    return 0.5 * ((I1 - J) ** 2).sum() + lam * (normV + rho * (p0 ** 2).sum())


def cost_and_grad(S, J, p0, rho, sigma, lam, T):
    S = torch.as_tensor(S, dtype=torch.float64)
    J = torch.as_tensor(J, dtype=torch.float64)
    p = torch.as_tensor(p0, dtype=torch.float64).clone().requires_grad_(True)
    H = cost(S, J, p, float(rho), float(sigma), float(lam), int(T))
    H.backward()
    return float(H.detach()), p.grad.numpy()
