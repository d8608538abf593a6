"""Seeded synthetic inputs for the multi-block structured-grid solver.

This module builds what both the GPU library and the CPU oracle take as
input, and nothing else: node coordinates per block, the block-to-block
connection table, the physical boundary table, flow parameters and the
initial conserved state at cell centroids.  It contains none of the solver's
arithmetic (no metrics, no fluxes, no ghost fill, no time stepping).

Conventions shared by every consumer
------------------------------------
* Directions d = 0, 1, 2 are the index directions i, j, k.
* Faces 0..5 are -i, +i, -j, +j, -k, +k (face = 2*d + side).
* A block of (ni, nj, nk) cells has nodes ``[3, nk+1, nj+1, ni+1]`` and an
  interior state ``[5, nk, nj, ni]`` (i fastest), components
  (rho, rho*u, rho*v, rho*w, rho*E) as in the paper's Eq. (1).
* Patch ranges on a face are given in the two transverse directions in
  ascending order (i-face: (j, k); j-face: (i, k); k-face: (i, j)), as
  half-open cell ranges ``lo <= p < hi``.
* A connection fills the ghost cells of ``face`` of ``blk`` from the cells of
  ``nbr`` just inside ``nbr_face``; only opposite faces of the same direction
  are connected (identity orientation).  Transverse index p on this block maps
  to ``p - lo + nbr_lo`` on the neighbour.  ``shift`` is added to the
  neighbour's node coordinates (periodic translation), else zero.
* Index space must be right-handed: (x(i), x(j), x(k)) forms a positive
  frame, so that face vectors point towards increasing index.

Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Sequence, Tuple

import numpy as np

FARFIELD, SLIPWALL, NOSLIP_ADIABATIC, EXTRAP = 1, 2, 3, 4
BC_NAMES = {FARFIELD: "farfield", SLIPWALL: "slipwall",
            NOSLIP_ADIABATIC: "noslip_adiabatic", EXTRAP: "extrapolate"}
NGHOST = 2

# Limiter constant of the steady channel marches.  The smooth limiter
# (2ab + eps) / (a^2 + b^2 + eps) of two one-sided differences a, b is 1 (no
# limiting) where both are well below sqrt(eps) and the plain ratio where both
# are well above.  With 1e-12 it flips between those limits at near-uniform
# faces from one step to the next and the transonic marches stall at a
# residual drop of about 6e-3; with 1e-4 (differences below about 1e-2 left
# unlimited) every case converges linearly.
STEADY_LIMITER_EPS = 1.0e-4


@dataclass
class Params:
    gamma: float = 1.4
    prandtl: float = 0.72
    mach: float = 0.5
    alpha: float = 0.0          # flow angle in the x-y plane [rad]
    beta: float = 0.0           # flow angle out of the x-y plane [rad]
    reynolds: float = 1.0e6     # per unit length, based on rho_inf, |u_inf|
    sutherland: float = 110.4 / 288.15
    cfl: float = 0.5
    entropy_fix: float = 0.1
    limiter_eps: float = 1.0e-12
    viscous: int = 0
    flux_fp32: int = 0
    local_dt: int = 0
    ghost_layers: int = NGHOST


@dataclass
class Conn:
    blk: int
    face: int
    nbr: int
    nbr_face: int
    lo: Tuple[int, int]
    hi: Tuple[int, int]
    nbr_lo: Tuple[int, int]
    shift: Tuple[float, float, float] = (0.0, 0.0, 0.0)


@dataclass
class BC:
    blk: int
    face: int
    kind: int
    lo: Tuple[int, int]
    hi: Tuple[int, int]
    mach: float = 0.0   # far field: this patch's freestream Mach (<= 0: the case's)


@dataclass
class Case:
    name: str
    params: Params
    dims: List[Tuple[int, int, int]]
    nodes: List[np.ndarray]
    conns: List[Conn]
    bcs: List[BC]
    q0: List[np.ndarray]
    info: dict = field(default_factory=dict)

    @property
    def nblk(self) -> int:
        return len(self.dims)

    @property
    def ncells(self) -> int:
        return int(sum(a * b * c for a, b, c in self.dims))

    def with_params(self, **kw) -> "Case":
        return replace(self, params=replace(self.params, **kw))


def transverse(d: int) -> Tuple[int, int]:
    """The two directions other than d, ascending."""
    return tuple(t for t in range(3) if t != d)  # type: ignore[return-value]


def face_extent(dims: Sequence[int], face: int) -> Tuple[int, int]:
    t1, t2 = transverse(face // 2)
    return dims[t1], dims[t2]


# --------------------------------------------------------------------------
# initial state helpers (input preparation only)

def freestream_velocity(p: Params) -> np.ndarray:
    speed = p.mach * math.sqrt(p.gamma)     # c_inf = sqrt(gamma * p/rho) = sqrt(gamma)
    return speed * np.array([math.cos(p.alpha) * math.cos(p.beta),
                             math.sin(p.alpha) * math.cos(p.beta),
                             math.sin(p.beta)])


def centroids(nodes):
    """Mean of the 8 corner nodes of every cell: [3, nk, nj, ni] (NumPy or torch)."""
    x = nodes
    c = x[:, :-1, :-1, :-1] + x[:, :-1, :-1, 1:]
    c += x[:, :-1, 1:, :-1]
    c += x[:, :-1, 1:, 1:]
    c += x[:, 1:, :-1, :-1]
    c += x[:, 1:, :-1, 1:]
    c += x[:, 1:, 1:, :-1]
    c += x[:, 1:, 1:, 1:]
    c *= 0.125
    return c


def conserved_from(rho, u, v, w, p, gamma):
    """Conserved variables [5, ...] from primitives; u, v, w may be scalars
    (a uniform velocity).  NumPy, or torch for device-generated inputs."""
    if isinstance(rho, np.ndarray):
        q = np.empty((5,) + rho.shape)
    else:
        import torch
        q = torch.empty((5,) + tuple(rho.shape), dtype=torch.float64, device=rho.device)
    q[0] = rho
    q[1] = rho * u
    q[2] = rho * v
    q[3] = rho * w
    q[4] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return q


def uniform_state(dims, p: Params) -> np.ndarray:
    ni, nj, nk = dims
    uvw = freestream_velocity(p)
    one = np.ones((nk, nj, ni))
    return conserved_from(one, uvw[0] * one, uvw[1] * one, uvw[2] * one, one, p.gamma)


# --------------------------------------------------------------------------
# grid helpers

def cartesian_nodes(dims, origin=(0.0, 0.0, 0.0), h=(1.0, 1.0, 1.0)) -> np.ndarray:
    ni, nj, nk = dims
    i = np.arange(ni + 1, dtype=np.float64)
    j = np.arange(nj + 1, dtype=np.float64)
    k = np.arange(nk + 1, dtype=np.float64)
    K, J, I = np.meshgrid(k, j, i, indexing="ij")
    return np.stack([origin[0] + h[0] * I, origin[1] + h[1] * J, origin[2] + h[2] * K])


def periodic_self_conns(blk: int, dims, lengths) -> List[Conn]:
    """Periodic self-connection on every face of a block."""
    out = []
    for d in range(3):
        t1, t2 = transverse(d)
        hi = (dims[t1], dims[t2])
        sh = [0.0, 0.0, 0.0]
        sh[d] = -lengths[d]
        out.append(Conn(blk, 2 * d, blk, 2 * d + 1, (0, 0), hi, (0, 0), tuple(sh)))
        sh = [0.0, 0.0, 0.0]
        sh[d] = lengths[d]
        out.append(Conn(blk, 2 * d + 1, blk, 2 * d, (0, 0), hi, (0, 0), tuple(sh)))
    return out


def periodic_pair(blk: int, dims, d: int, length: float) -> List[Conn]:
    t1, t2 = transverse(d)
    hi = (dims[t1], dims[t2])
    sm = [0.0, 0.0, 0.0]
    sm[d] = -length
    sp = [0.0, 0.0, 0.0]
    sp[d] = length
    return [Conn(blk, 2 * d, blk, 2 * d + 1, (0, 0), hi, (0, 0), tuple(sm)),
            Conn(blk, 2 * d + 1, blk, 2 * d, (0, 0), hi, (0, 0), tuple(sp))]


def full_bc(blk: int, dims, face: int, kind: int) -> BC:
    return BC(blk, face, kind, (0, 0), face_extent(dims, face))


# --------------------------------------------------------------------------
# workloads

def isentropic_vortex_primitives(x, y, xc, yc, p: Params, strength=5.0, radius=1.0,
                                 period=None):
    """Isentropic vortex on the uniform stream (rho = p = 1, T = p/rho)."""
    g = p.gamma
    dx = x - xc
    dy = y - yc
    if period is not None:
        dx = dx - period * np.round(dx / period)
        dy = dy - period * np.round(dy / period)
    r2 = (dx * dx + dy * dy) / (radius * radius)
    f = np.exp(0.5 * (1.0 - r2))
    uinf = freestream_velocity(p)
    u = uinf[0] - strength / (2.0 * math.pi) * dy / radius * f
    v = uinf[1] + strength / (2.0 * math.pi) * dx / radius * f
    w = uinf[2] + 0.0 * x
    T = 1.0 - (g - 1.0) * strength ** 2 / (8.0 * g * math.pi ** 2) * f * f
    rho = T ** (1.0 / (g - 1.0))
    return rho, u, v, w, rho * T


def vortex_case(n: int = 32, seed: int = 0, nz: int | None = None, mach: float = 0.5,
                cfl: float = 0.5, curvilinear: bool = False, half: float = 5.0) -> Case:
    """3-D Euler isentropic vortex in a periodic box [-half, half]^3.

    One block of n x n x nz cells, periodic on all faces; vortex strength 5,
    radius 1, centre offset drawn from the seed.  ``curvilinear`` applies a
    smooth periodic node displacement (amplitude 0.4 h) so that metrics are
    non-trivial while periodicity is kept.
    """
    nz = n if nz is None else nz
    rng = np.random.default_rng(seed)
    xc, yc = rng.uniform(-1.0, 1.0, 2)
    L = 2.0 * half
    h = L / n
    hz = L / nz
    dims = (n, n, nz)
    X = cartesian_nodes(dims, origin=(-half, -half, -half), h=(h, h, hz))
    if curvilinear:
        a = 0.4 * h
        kx = 2.0 * math.pi / L
        x0, y0, z0 = X[0].copy(), X[1].copy(), X[2].copy()
        X[0] = x0 + a * np.sin(kx * y0) * np.sin(kx * z0)
        X[1] = y0 + a * np.sin(kx * x0) * np.sin(kx * z0)
        X[2] = z0 + a * np.sin(kx * x0) * np.sin(kx * y0)
    par = Params(mach=mach, cfl=cfl, viscous=0)
    C = centroids(X)
    rho, u, v, w, pr = isentropic_vortex_primitives(C[0], C[1], xc, yc, par, period=L)
    q = conserved_from(rho, u, v, w, pr, par.gamma)
    return Case("vortex", par, [dims], [X], periodic_self_conns(0, dims, (L, L, L)), [], [q],
                info={"xc": float(xc), "yc": float(yc), "period": L, "seed": seed})


def bump_wall_y(x, z, amp):
    return amp * np.sin(0.5 * math.pi * x) ** 2 * (0.75 + 0.25 * np.cos(2.0 * math.pi * z))


def bump_ns_case(ni: int = 256, nj: int = 128, nk: int = 128, seed: int = 0, mach: float = 0.8,
                 reynolds: float = 1.0e6, noise: float = 1.0e-3, stretch: float = 2.0,
                 amp: float = 0.05, viscous: int = 1, cfl: float = 0.5) -> Case:
    """Compressible Navier-Stokes over a sinusoidal wall bump, one curvilinear block.

    i = x in [0, 2] (periodic), j = wall-normal (no-slip adiabatic wall at
    j = 0, far field at j = nj) with tanh stretching, k = z in [0, 1]
    (periodic).  Freestream plus seeded uniform noise of relative size
    ``noise`` on every conserved variable.
    """
    rng = np.random.default_rng(seed)
    dims = (ni, nj, nk)
    i = np.arange(ni + 1) / ni * 2.0
    eta = np.arange(nj + 1) / nj
    z = np.arange(nk + 1) / nk
    K, J, I = np.meshgrid(z, eta, i, indexing="ij")
    yw = bump_wall_y(I, K, amp)
    t = 1.0 + np.tanh(stretch * (J - 1.0)) / math.tanh(stretch)
    Y = yw + (1.0 - yw) * t
    X = np.stack([I, Y, K]).astype(np.float64)
    par = Params(mach=mach, reynolds=reynolds, viscous=viscous, cfl=cfl)
    q = uniform_state(dims, par)
    uinf = freestream_velocity(par)
    speed = float(np.linalg.norm(uinf))
    e_inf = 1.0 / (par.gamma - 1.0) + 0.5 * speed ** 2
    qref = np.array([1.0, speed, speed, speed, e_inf])
    q = q + noise * rng.uniform(-1.0, 1.0, q.shape) * qref[:, None, None, None]
    conns = periodic_pair(0, dims, 0, 2.0) + periodic_pair(0, dims, 2, 1.0)
    bcs = [full_bc(0, dims, 2, NOSLIP_ADIABATIC), full_bc(0, dims, 3, FARFIELD)]
    return Case("bump_ns", par, [dims], [X], conns, bcs, [q], info={"seed": seed})


def pressure_pulses(C, centres, amp, sigma, par: Params):
    """Isentropic Gaussian pressure pulses on the uniform stream.

    C: cell centres [3, ...] (NumPy or torch).  A pulse whose exponent exceeds
    750 at every cell (judged from the box bounding C) contributes exactly
    0.0 in FP64 (exp underflows), so it is skipped: the sum is bitwise the
    full one."""
    xp = _xp(C)
    s = xp.zeros(C.shape[1:], dtype=C.dtype, **_dev_kw(C))
    lo = [float(C[a].min()) for a in range(3)]
    hi = [float(C[a].max()) for a in range(3)]
    for c in centres:
        d2 = sum(max(0.0, lo[a] - c[a], c[a] - hi[a]) ** 2 for a in range(3))
        if d2 / (2.0 * sigma * sigma) > 750.0:
            continue
        r2 = (C[0] - c[0]) ** 2 + (C[1] - c[1]) ** 2 + (C[2] - c[2]) ** 2
        s = s + xp.exp(-r2 / (2.0 * sigma * sigma))
    pr = 1.0 + amp * s
    rho = pr ** (1.0 / par.gamma)
    uinf = freestream_velocity(par)
    return conserved_from(rho, float(uinf[0]), float(uinf[1]), float(uinf[2]), pr, par.gamma)


def _xp(a):
    """The array module of a (NumPy, or torch for device-generated inputs)."""
    if isinstance(a, np.ndarray):
        return np
    import torch
    return torch


def _dev_kw(a):
    return {} if isinstance(a, np.ndarray) else {"device": a.device}


def batched_euler_case(nblk: int = 64, seed: int = 0, lo: int = 16, hi: int = 161,
                       mach: float = 0.5, flux_fp32: int = 1, cfl: float = 0.5,
                       h: float | None = None) -> Case:
    """Many uneven curvilinear Euler blocks joined in a seeded chain.

    Block dims are drawn uniformly in [lo, hi).  A seeded permutation orders
    the blocks; block n's +i face connects to block n+1's -i face over the
    overlap rectangle anchored at the face origin, and every other boundary
    cell face is far field.  Blocks sit side by side in x on one global
    uniform lattice (spacing h, default 1/64) displaced by a smooth global
    mapping (amplitude 2h, wavelength 32h), so nodes match bitwise across
    the chain.  Eight seeded isentropic Gaussian pressure pulses (amplitude
    1e-2, sigma 8h) ride on the Mach ``mach`` stream.
    """
    rng = np.random.default_rng(seed)
    dims_arr = rng.integers(lo, hi, (nblk, 3))
    order = rng.permutation(nblk)
    h = 1.0 / 64.0 if h is None else h
    A, lam = 2.0 * h, 32.0 * h
    dims = [tuple(int(v) for v in dims_arr[b]) for b in range(nblk)]
    xoff = {}
    acc = 0
    for b in order:
        xoff[int(b)] = acc
        acc += dims[int(b)][0]
    par = Params(mach=mach, viscous=0, flux_fp32=flux_fp32, cfl=cfl)
    nodes = []
    w = 2.0 * math.pi / lam
    for b in range(nblk):
        ni, nj, nk = dims[b]
        # x, y, z are each a function of one index; the mapping's sines are
        # evaluated once per index and broadcast (the same bits as on the
        # full lattice)
        x = ((np.arange(ni + 1) + xoff[b]) * h)[None, None, :]
        y = (np.arange(nj + 1) * h)[None, :, None]
        z = (np.arange(nk + 1) * h)[:, None, None]
        sx, sy, sz = np.sin(w * x), np.sin(w * y), np.sin(w * z)
        X = np.empty((3, nk + 1, nj + 1, ni + 1))
        X[0] = x + A * sy * sz
        X[1] = y + A * sx * sz
        X[2] = z + A * sx * sy
        nodes.append(X)
    ymax = max(d[1] for d in dims) * h
    zmax = max(d[2] for d in dims) * h
    centres = np.column_stack([rng.uniform(0.0, acc * h, 8), rng.uniform(0.0, ymax, 8),
                               rng.uniform(0.0, zmax, 8)])
    q0 = [pressure_pulses(centroids(nodes[b]), centres, 1e-2, 8.0 * h, par) for b in range(nblk)]
    conns: List[Conn] = []
    bcs: List[BC] = []
    covered = {}
    for n in range(nblk - 1):
        a, b = int(order[n]), int(order[n + 1])
        mj = min(dims[a][1], dims[b][1])
        mk = min(dims[a][2], dims[b][2])
        conns.append(Conn(a, 1, b, 0, (0, 0), (mj, mk), (0, 0)))
        conns.append(Conn(b, 0, a, 1, (0, 0), (mj, mk), (0, 0)))
        covered[(a, 1)] = (mj, mk)
        covered[(b, 0)] = (mj, mk)
    for b in range(nblk):
        for face in range(6):
            e1, e2 = face_extent(dims[b], face)
            if (b, face) not in covered:
                bcs.append(BC(b, face, FARFIELD, (0, 0), (e1, e2)))
                continue
            mj, mk = covered[(b, face)]
            if e1 > mj:
                bcs.append(BC(b, face, FARFIELD, (mj, 0), (e1, e2)))
            if e2 > mk:
                bcs.append(BC(b, face, FARFIELD, (0, mk), (mj, e2)))
    return Case("batched_euler", par, dims, nodes, conns, bcs, q0,
                info={"seed": seed, "order": [int(v) for v in order]})


def channel_bump_wall_y(x, z, hb):
    inside = (x >= 0.5) & (x <= 1.5)
    return np.where(inside, hb * np.sin(math.pi * (x - 0.5)) ** 2
                    * (0.75 + 0.25 * np.cos(2.0 * math.pi * z)), 0.0)


def channel_nodes(ni, nj, nk, hb):
    x = np.arange(ni + 1) / ni * 2.0
    eta = np.arange(nj + 1) / nj
    z = np.arange(nk + 1) / nk
    K, J, I = np.meshgrid(z, eta, x, indexing="ij")
    yw = channel_bump_wall_y(I, K, hb)
    Y = yw + (1.0 - yw) * J
    return np.stack([I, Y, K]).astype(np.float64)


def channel_case(ni: int, nj: int, nk: int, mach: float, hb: float, cfl: float = 1.0,
                 local_dt: int = 1, limiter_eps: float = STEADY_LIMITER_EPS) -> Case:
    """Steady inviscid channel with a wall bump (learned warm-start workload).

    x in [0, 2] with far-field inflow/outflow on the i faces, slip walls on
    both j faces (bump of height hb on the lower wall for 0.5 <= x <= 1.5),
    z in [0, 1] periodic.  Starts from the uniform stream.
    """
    dims = (ni, nj, nk)
    X = channel_nodes(ni, nj, nk, hb)
    par = Params(mach=mach, viscous=0, cfl=cfl, local_dt=local_dt, limiter_eps=limiter_eps)
    q = uniform_state(dims, par)
    conns = periodic_pair(0, dims, 2, 1.0)
    bcs = [full_bc(0, dims, 0, FARFIELD), full_bc(0, dims, 1, FARFIELD),
           full_bc(0, dims, 2, SLIPWALL), full_bc(0, dims, 3, SLIPWALL)]
    return Case("channel", par, [dims], [X], conns, bcs, [q], info={"mach": mach, "hb": hb})


def channel_batch_case(conds, ni: int = 48, nj: int = 24, nk: int = 24, cfl: float = 1.0,
                       local_dt: int = 1, limiter_eps: float = STEADY_LIMITER_EPS) -> Case:
    """Independent channel-bump cases side by side, one block each.

    ``conds[b] = (inflow Mach, bump height)``.  Each block is its own channel
    (periodic in z onto itself, far field on the i faces carrying that block's
    Mach number, slip walls on the j faces) starting from its own uniform
    stream, so one context advances all cases at once.
    """
    dims_b = (ni, nj, nk)
    par = Params(mach=float(conds[0][0]), viscous=0, cfl=cfl, local_dt=local_dt, limiter_eps=limiter_eps)
    dims, nodes, q0, conns, bcs = [], [], [], [], []
    for b, (m, hb) in enumerate(conds):
        dims.append(dims_b)
        nodes.append(channel_nodes(ni, nj, nk, float(hb)))
        q0.append(uniform_state(dims_b, replace(par, mach=float(m))))
        conns += periodic_pair(b, dims_b, 2, 1.0)
        for face, kind in ((0, FARFIELD), (1, FARFIELD), (2, SLIPWALL), (3, SLIPWALL)):
            bc = full_bc(b, dims_b, face, kind)
            bc.mach = float(m) if kind == FARFIELD else 0.0
            bcs.append(bc)
    return Case("channel_batch", par, dims, nodes, conns, bcs, q0,
                info={"conds": [(float(m), float(h)) for m, h in conds]})


def mlp_init(d_in: int = 5, d_hidden: int = 128, n_hidden: int = 4, d_out: int = 5, seed: int = 0,
             out_scale: float = 0.1):
    """Seeded initial weights of the warm-start network: list of (W [out, in], b [out]).

    Glorot-uniform weights, zero biases; the output layer is scaled by
    ``out_scale`` so the initial prediction is close to the inflow stream.
    """
    rng = np.random.default_rng(seed)
    sizes = [d_in] + [d_hidden] * n_hidden + [d_out]
    out = []
    for l in range(len(sizes) - 1):
        fi, fo = sizes[l], sizes[l + 1]
        a = math.sqrt(6.0 / (fi + fo))
        W = rng.uniform(-a, a, (fo, fi))
        if l == len(sizes) - 2:
            W = W * out_scale
        out.append((W, np.zeros(fo)))
    return out


def channel_conditions(n: int, seed: int) -> np.ndarray:
    """Inflow Mach in [0.5, 0.85) and bump height in [0.02, 0.1) per case,
    drawn a pair at a time: the first k cases are the same for every n >= k."""
    u = np.random.default_rng(seed).uniform(size=(n, 2))
    return np.column_stack([0.5 + 0.35 * u[:, 0], 0.02 + 0.08 * u[:, 1]])


class LazyStates:
    """Initial states computed block by block when read (device-generated
    workloads whose states do not all fit in memory at once)."""

    def __init__(self, n, make):
        self._n = n
        self._make = make

    def __len__(self):
        return self._n

    def __getitem__(self, b):
        if not 0 <= b < self._n:
            raise IndexError(b)
        return self._make(b)

    def __iter__(self):
        return (self._make(b) for b in range(self._n))


def paper_share_case(nbx: int = 4, nbz: int = 4, ni: int = 512, nj: int = 512, nk: int = 144,
                     seed: int = 0, mach: float = 0.8, reynolds: float = 1.0e6,
                     flux_fp32: int = 1, viscous: int = 1, amp: float = 0.05,
                     stretch: float = 2.0, pulses: bool = True, cfl: float = 0.5, log=None,
                     device=None) -> Case:
    """One GPU's share of a large multi-block wall-bounded flow.

    nbx x nbz blocks tile x in [0, nbx] and z in [0, nbz], each block one
    unit square in x-z; index directions are i = z, j = x, k = wall-normal
    (a right-handed frame).  The lower k face is a no-slip adiabatic wall
    with a sinusoidal bump, the upper k face is far field at y = 1, and the
    outer x and z faces are periodic.  Eight seeded isentropic Gaussian
    pressure pulses (amplitude 1e-2, sigma 0.1) ride on the stream.  log, if
    given, is called with a progress line after every block.

    device (e.g. "cuda:0"): the same recipe evaluated with torch on that
    device; nodes are device tensors and the initial states a LazyStates
    (each block's state computed from its nodes when read), so the 604 M
    cell workload is generated in seconds without host memory.  The device's
    sin/tanh/exp may round differently from NumPy's, so the two paths agree
    to rounding, not bitwise; parity tests use the NumPy path for both sides.
    """
    rng = np.random.default_rng(seed)
    par = Params(mach=mach, reynolds=reynolds, viscous=viscous, flux_fp32=flux_fp32, cfl=cfl)
    Lx, Lz = float(nbx), float(nbz)
    centres = np.column_stack([rng.uniform(0.0, Lx, 8), rng.uniform(0.2, 0.8, 8),
                               rng.uniform(0.0, Lz, 8)])
    if device is not None:
        import torch
        xp = torch
        kw = {"dtype": torch.float64, "device": torch.device(device)}
    else:
        xp = np
        kw = {"dtype": np.float64}
    dims, nodes, q0 = [], [], []
    bid = {}
    for bx in range(nbx):
        for bz in range(nbz):
            bid[(bx, bz)] = len(dims)
            zz = bz + xp.arange(ni + 1, **kw) / ni
            xx = bx + xp.arange(nj + 1, **kw) / nj
            eta = xp.arange(nk + 1, **kw) / nk
            E, Xg, Zg = xp.meshgrid(eta, xx, zz, indexing="ij")
            yw = amp * xp.sin(math.pi * Xg) ** 2 * (0.75 + 0.25 * xp.cos(2.0 * math.pi * Zg))
            t = 1.0 + xp.tanh(stretch * (E - 1.0)) / math.tanh(stretch)
            Y = yw + (1.0 - yw) * t
            X = xp.stack([Xg, Y, Zg])
            if device is None:
                X = X.astype(np.float64, copy=False)
            dims.append((ni, nj, nk))
            nodes.append(X)
            if device is None:
                if pulses:
                    q0.append(pressure_pulses(centroids(X), centres, 1e-2, 0.1, par))
                else:
                    q0.append(uniform_state((ni, nj, nk), par))
            if log:
                log(f"# block {len(dims)}/{nbx * nbz} generated")
    if device is not None:
        def make(b, nodes=nodes):
            if pulses:
                return pressure_pulses(centroids(nodes[b]), centres, 1e-2, 0.1, par)
            import torch
            return torch.from_numpy(uniform_state((ni, nj, nk), par)).to(nodes[b].device)
        q0 = LazyStates(len(dims), make)
    conns, bcs = [], []
    for bx in range(nbx):
        for bz in range(nbz):
            b = bid[(bx, bz)]
            # i = z direction
            up = bid[(bx, (bz + 1) % nbz)]
            dn = bid[(bx, (bz - 1) % nbz)]
            shp = (0.0, 0.0, Lz if bz == nbz - 1 else 0.0)
            shm = (0.0, 0.0, -Lz if bz == 0 else 0.0)
            conns.append(Conn(b, 1, up, 0, (0, 0), (nj, nk), (0, 0), shp))
            conns.append(Conn(b, 0, dn, 1, (0, 0), (nj, nk), (0, 0), shm))
            # j = x direction
            up = bid[((bx + 1) % nbx, bz)]
            dn = bid[((bx - 1) % nbx, bz)]
            shp = (Lx if bx == nbx - 1 else 0.0, 0.0, 0.0)
            shm = (-Lx if bx == 0 else 0.0, 0.0, 0.0)
            conns.append(Conn(b, 3, up, 2, (0, 0), (ni, nk), (0, 0), shp))
            conns.append(Conn(b, 2, dn, 3, (0, 0), (ni, nk), (0, 0), shm))
            bcs.append(BC(b, 4, NOSLIP_ADIABATIC, (0, 0), (ni, nj)))
            bcs.append(BC(b, 5, FARFIELD, (0, 0), (ni, nj)))
    return Case("paper_share", par, dims, nodes, conns, bcs, q0, info={"seed": seed})


def paper_share_vertices(nbx: int = 4, nbz: int = 4, ni: int = 512, nj: int = 512, nk: int = 144,
                         amp: float = 0.05, stretch: float = 2.0):
    """The whole grid of paper_share_case (its nbx x nbz blocks side by side)
    as the vertex array of the WCNS-E-5 closures: index i = z and j = x
    periodic (their nbz ni and nbx nj upper corners), k = wall-normal with its
    nk + 1 vertex planes (the wall first).  Returns (Xv [3, nk + 1, nbx nj,
    nbz ni], period [3][3]); vertex (i, j, k) sits where paper_share_case puts
    node (i + 1, j + 1, k) of the whole grid."""
    NI, NJ = nbz * ni, nbx * nj
    zz = (np.arange(NI) + 1.0) / ni
    xx = (np.arange(NJ) + 1.0) / nj
    eta = np.arange(nk + 1) / nk
    E, Xg, Zg = np.meshgrid(eta, xx, zz, indexing="ij")
    yw = amp * np.sin(math.pi * Xg) ** 2 * (0.75 + 0.25 * np.cos(2.0 * math.pi * Zg))
    t = 1.0 + np.tanh(stretch * (E - 1.0)) / math.tanh(stretch)
    Y = yw + (1.0 - yw) * t
    period = [(0.0, 0.0, float(nbz)), (float(nbx), 0.0, 0.0), (0.0, 0.0, 0.0)]
    return np.stack([Xg, Y, Zg]).astype(np.float64), period


def coarsen_case(case: Case) -> Case:
    """The next coarser grid of a multigrid hierarchy: every block keeps every
    second node along each direction (the coarse cells are unions of 2 x 2 x 2
    fine cells, nested exactly), and the connection and boundary tables keep
    their patches with every range halved.  Every extent and patch bound must
    be even.  The initial state is the uniform stream (a cycle overwrites it
    with the restricted fine state)."""
    dims, nodes = [], []
    for (ni, nj, nk), X in zip(case.dims, case.nodes):
        if ni % 2 or nj % 2 or nk % 2:
            raise ValueError(f"block extents {ni, nj, nk} are not all even")
        dims.append((ni // 2, nj // 2, nk // 2))
        nodes.append(np.ascontiguousarray(X[:, ::2, ::2, ::2]))

    def half(v):
        if any(x % 2 for x in v):
            raise ValueError(f"patch bound {v} is not even")
        return tuple(x // 2 for x in v)
    conns = [replace(c, lo=half(c.lo), hi=half(c.hi), nbr_lo=half(c.nbr_lo)) for c in case.conns]
    bcs = [replace(b, lo=half(b.lo), hi=half(b.hi)) for b in case.bcs]
    q0 = [uniform_state(d, case.params) for d in dims]
    return Case(case.name + "_coarse", case.params, dims, nodes, conns, bcs, q0, dict(case.info))


def hierarchy(case: Case, nlevels: int) -> List[Case]:
    """[case, its coarsening, ...], nlevels grids."""
    out = [case]
    for _ in range(nlevels - 1):
        out.append(coarsen_case(out[-1]))
    return out


def split_periodic_box(case: Case, parts=(2, 2, 2)) -> Case:
    """Split a single periodic block into parts[0] x parts[1] x parts[2] blocks.

    The split blocks are joined by 1-to-1 connections (the outer ones carry
    the periodic shift), and node coordinates and states are sliced from the
    parent, so both describe the same discrete problem.
    """
    assert case.nblk == 1
    ni, nj, nk = case.dims[0]
    pi, pj, pk = parts
    assert ni % pi == 0 and nj % pj == 0 and nk % pk == 0
    si, sj, sk = ni // pi, nj // pj, nk // pk
    X = case.nodes[0]
    Q = case.q0[0]
    lengths = []
    for d in range(3):
        for c in case.conns:
            if c.face == 2 * d + 1:
                lengths.append(c.shift[d])
                break
    dims, nodes, q0, bid = [], [], [], {}
    for bk in range(pk):
        for bj in range(pj):
            for bi in range(pi):
                bid[(bi, bj, bk)] = len(dims)
                dims.append((si, sj, sk))
                nodes.append(X[:, bk * sk:(bk + 1) * sk + 1, bj * sj:(bj + 1) * sj + 1,
                               bi * si:(bi + 1) * si + 1].copy())
                q0.append(Q[:, bk * sk:(bk + 1) * sk, bj * sj:(bj + 1) * sj,
                            bi * si:(bi + 1) * si].copy())
    conns = []
    P = (pi, pj, pk)
    sub = (si, sj, sk)
    for (bi, bj, bk), b in bid.items():
        idx = [bi, bj, bk]
        for d in range(3):
            t1, t2 = transverse(d)
            hi = (sub[t1], sub[t2])
            for side in (0, 1):
                nidx = list(idx)
                step = 1 if side else -1
                nidx[d] = (idx[d] + step) % P[d]
                sh = [0.0, 0.0, 0.0]
                if side == 1 and idx[d] == P[d] - 1:
                    sh[d] = lengths[d]
                if side == 0 and idx[d] == 0:
                    sh[d] = -lengths[d]
                conns.append(Conn(b, 2 * d + side, bid[tuple(nidx)], 2 * d + 1 - side,
                                  (0, 0), hi, (0, 0), tuple(sh)))
    return Case(case.name + "_split", case.params, dims, nodes, conns, [], q0, dict(case.info))
