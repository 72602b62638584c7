"""Seeded synthetic convection-diffusion-reaction (CDR) instances on the unit cube.

This module is the input side shared by the GPU path and the CPU oracle.  It
produces the Galerkin finite element data of the paper's semi-discrete problem
(Sec. 2, eqs. (2)-(4)): the consistent mass matrix M_C, the transport operator
K = -A (A = diffusion + convection + reaction), its convective part
K_conv = -C (the eps = 0, c = 0 operator that the monolithic convex limiter is
applied to, Remark 1 in Sec. 2.2), the load vector F, the Dirichlet set with
its values, and initial states.  It holds none of the algebraic flux correction
arithmetic: no lumping, no artificial diffusion, no fluxes, no limiter, no
solver.

Meshes (the paper refines cube meshes uniformly, Sec. 4):
  * Q1: n^3 cubes of edge h = 1/n, (n+1)^3 nodes, 27-point rows.
  * P1: every cube split into 6 Kuhn tetrahedra along its main diagonal
    (a conforming triangulation), 15-point rows.
Node numbering is lexicographic, index = ix + (n+1)*(iy + (n+1)*iz).  CSR rows
are sorted, contain the diagonal, and all matrices share one structurally
symmetric pattern: the support of M_C, i.e. N_i = {j : m_ij != 0} (eq. (23)).

Quadrature: Q1 matrices are Kronecker products of exact 1D integrals (three
point Gauss per cell) and are exact for constant eps, c and affine b.  P1
matrices use the closed forms for linear elements, exact for affine b.

Random draws use numpy.random.default_rng((0, config_id, k)).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------
# Instance container
# ----------------------------------------------------------------------------


@dataclass
class Instance:
    """One CDR problem on a fixed mesh.

    row_ptr/col: int32 CSR pattern (N+1, nnz).  M, K, K_conv: float64 values on
    that pattern.  F: load vector.  dir_idx/dir_val: Dirichlet nodes (sorted
    int32) and their values.  u0: initial state (time-dependent problems).
    """

    elem: str
    n: int
    N: int
    row_ptr: np.ndarray
    col: np.ndarray
    M: np.ndarray
    K: np.ndarray
    K_conv: np.ndarray
    F: np.ndarray
    dir_idx: np.ndarray
    dir_val: np.ndarray
    u0: np.ndarray
    coords: np.ndarray
    params: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def row_index(self) -> np.ndarray:
        return np.repeat(np.arange(self.N, dtype=np.int64), np.diff(self.row_ptr))


# ----------------------------------------------------------------------------
# Velocity fields: b(x) = b0 + B x
# ----------------------------------------------------------------------------


def affine_field(b0, B=None):
    b0 = np.asarray(b0, dtype=np.float64).reshape(3)
    B = np.zeros((3, 3)) if B is None else np.asarray(B, dtype=np.float64).reshape(3, 3)
    return b0, B


def eval_field(field_, X):
    b0, B = field_
    return b0[None, :] + X @ B.T


ROTATING_B = affine_field([0.5, -0.5, 0.1], [[0, -1, 0], [1, 0, 0], [0, 0, 0]])
"""b = (-(y - 1/2), x - 1/2, 0.1): rotation about the axis x = y = 1/2 plus a lift."""


def grid_coords(n: int) -> np.ndarray:
    h = 1.0 / n
    i = np.arange(n + 1, dtype=np.float64) * h
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


# ----------------------------------------------------------------------------
# Q1: tensor-product assembly
# ----------------------------------------------------------------------------

_GAUSS3_T = np.array([0.5 - math.sqrt(0.6) / 2, 0.5, 0.5 + math.sqrt(0.6) / 2])
_GAUSS3_W = np.array([5.0, 8.0, 5.0]) / 18.0


def _band_1d(n: int, trial_deriv: bool, test_deriv: bool, weight_x: bool) -> np.ndarray:
    """1D integrals F[i, o+1] = int w(x) psi_{i+o} chi_i over [0, 1], o in {-1,0,1}.

    psi is the trial hat function (or its derivative), chi the test hat function
    (or its derivative), w(x) = x or 1.  Three-point Gauss per cell is exact for
    the degrees that occur here (<= 3).
    """
    h = 1.0 / n
    band = np.zeros((n + 1, 3))
    t = _GAUSS3_T
    w = _GAUSS3_W * h
    phi = [1.0 - t, t]
    dphi = [np.full(3, -1.0 / h), np.full(3, 1.0 / h)]
    for e in range(n):
        wx = (e * h + t * h) if weight_x else np.ones(3)
        for a in range(2):
            chi = dphi[a] if test_deriv else phi[a]
            for b_ in range(2):
                psi = dphi[b_] if trial_deriv else phi[b_]
                band[e + a, (b_ - a) + 1] += float(np.sum(w * wx * psi * chi))
    return band


_Q1_OFFSETS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _q1_pattern(n: int):
    """CSR pattern of the 27-point Q1 stencil, columns sorted."""
    m = n + 1
    N = m ** 3
    idx = np.arange(N, dtype=np.int64)
    ix, iy, iz = idx % m, (idx // m) % m, idx // (m * m)
    valid = np.empty((N, 27), dtype=bool)
    cols = np.empty((N, 27), dtype=np.int64)
    for o, (dx, dy, dz) in enumerate(_Q1_OFFSETS):
        jx, jy, jz = ix + dx, iy + dy, iz + dz
        valid[:, o] = (jx >= 0) & (jx < m) & (jy >= 0) & (jy < m) & (jz >= 0) & (jz < m)
        cols[:, o] = idx + dx + m * dy + m * m * dz
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[valid].astype(np.int32)
    return row_ptr.astype(np.int32), col, valid, (ix, iy, iz)


def _q1_values(n, valid, ijk, terms):
    """Values of sum_t coef_t * Fx_t (x) Fy_t (x) Fz_t on the pattern."""
    ix, iy, iz = ijk
    N = ix.shape[0]
    out = np.zeros((N, 27))
    for coef, (fx, fy, fz) in terms:
        for o, (dx, dy, dz) in enumerate(_Q1_OFFSETS):
            out[:, o] += coef * (fx[ix, dx + 1] * fy[iy, dy + 1] * fz[iz, dz + 1])
    return out[valid]


def _q1_operator_terms(n, eps, bfield, c):
    """Factor triples for M, the diffusion+reaction part E and the convective part C."""
    mass = _band_1d(n, False, False, False)
    stiff = _band_1d(n, True, True, False)
    deriv = _band_1d(n, True, False, False)
    mass_x = _band_1d(n, False, False, True)
    deriv_x = _band_1d(n, True, False, True)
    M_terms = [(1.0, (mass, mass, mass))]
    E_terms = []
    if eps != 0.0:
        E_terms += [(eps, (stiff, mass, mass)), (eps, (mass, stiff, mass)), (eps, (mass, mass, stiff))]
    if c != 0.0:
        E_terms += [(c, (mass, mass, mass))]
    b0, B = bfield
    C_terms = []
    for k in range(3):
        if b0[k] != 0.0:
            f = [deriv if d == k else mass for d in range(3)]
            C_terms.append((float(b0[k]), tuple(f)))
        for l_ in range(3):
            if B[k, l_] != 0.0:
                f = []
                for d in range(3):
                    if d == k:
                        f.append(deriv_x if d == l_ else deriv)
                    else:
                        f.append(mass_x if d == l_ else mass)
                C_terms.append((float(B[k, l_]), tuple(f)))
    return M_terms, E_terms, C_terms


def _box_load_1d(n, lo, hi):
    """int_{[lo,hi]} phi_i dx for the 1D hat functions (exact: linear integrand)."""
    h = 1.0 / n
    out = np.zeros(n + 1)
    for e in range(n):
        a, b = e * h, (e + 1) * h
        p, q = max(a, lo), min(b, hi)
        if q <= p:
            continue
        # two-point Gauss on [p, q] integrates the linear hats exactly
        for tg in (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)):
            x = p + tg * (q - p)
            wq = 0.5 * (q - p)
            out[e] += wq * (b - x) / h
            out[e + 1] += wq * (x - a) / h
    return out


# ----------------------------------------------------------------------------
# P1 (Kuhn tetrahedra): element assembly
# ----------------------------------------------------------------------------

_KUHN_PERMS = list(itertools.permutations(range(3)))
_P1_OFFSETS = sorted(
    {(dx, dy, dz) for dx in (0, 1) for dy in (0, 1) for dz in (0, 1)}
    | {(-dx, -dy, -dz) for dx in (0, 1) for dy in (0, 1) for dz in (0, 1)},
    key=lambda o: (o[2], o[1], o[0]),
)


def _kuhn_local_vertices():
    """Vertex offsets (4x3 ints) of the 6 Kuhn tetrahedra of the unit cube."""
    shapes = []
    for p in _KUHN_PERMS:
        v = [np.zeros(3, dtype=np.int64)]
        cur = np.zeros(3, dtype=np.int64)
        for k in p:
            cur = cur.copy()
            cur[k] = 1
            v.append(cur)
        shapes.append(np.stack(v))
    return shapes


def _p1_assemble(n, eps, bfield, c):
    m = n + 1
    N = m ** 3
    h = 1.0 / n
    cz, cy, cx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)  # (ncubes, 3)
    I_all, J_all = [], []
    Mv, Ev, Cv = [], [], []
    b0, B = bfield
    for verts in _kuhn_local_vertices():
        Xr = verts.astype(np.float64) * h  # local vertex coords (4,3)
        Jm = np.stack([Xr[1] - Xr[0], Xr[2] - Xr[0], Xr[3] - Xr[0]], axis=1)  # columns
        vol = abs(np.linalg.det(Jm)) / 6.0
        Jinv = np.linalg.inv(Jm)
        grads = np.zeros((4, 3))
        grads[1:] = Jinv  # row k-1 of J^{-1} is grad phi_k
        grads[0] = -grads[1:].sum(axis=0)
        mass_loc = vol / 20.0 * (np.ones((4, 4)) + np.eye(4))
        stiff_loc = vol * grads @ grads.T
        gidx = []
        Xg = []
        for a in range(4):
            p = base + verts[a][None, :]
            gidx.append(p[:, 0] + m * (p[:, 1] + m * p[:, 2]))
            Xg.append(p.astype(np.float64) * h)
        gidx = np.stack(gidx, axis=1)  # (ncubes, 4)
        bvert = np.stack([eval_field(bfield, X) for X in Xg], axis=1)  # (ncubes,4,3)
        bsum = bvert.sum(axis=1)  # (ncubes,3)
        for a in range(4):
            # int_T b phi_a = vol/20 * (sum_k b(x_k) + b(x_a)) for affine b
            bphi = vol / 20.0 * (bsum + bvert[:, a, :])  # (ncubes,3)
            for b_ in range(4):
                I_all.append(gidx[:, a])
                J_all.append(gidx[:, b_])
                Mv.append(np.full(gidx.shape[0], mass_loc[a, b_]))
                Ev.append(np.full(gidx.shape[0], eps * stiff_loc[a, b_] + c * mass_loc[a, b_]))
                Cv.append(bphi @ grads[b_])
    I = np.concatenate(I_all)
    J = np.concatenate(J_all)
    keys = I * N + J
    uniq, inv = np.unique(keys, return_inverse=True)
    nnz = uniq.shape[0]
    M = np.bincount(inv, weights=np.concatenate(Mv), minlength=nnz)
    E = np.bincount(inv, weights=np.concatenate(Ev), minlength=nnz)
    C = np.bincount(inv, weights=np.concatenate(Cv), minlength=nnz)
    rows = uniq // N
    col = (uniq % N).astype(np.int32)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=N), out=row_ptr[1:])
    return row_ptr.astype(np.int32), col, M, E, C


# ----------------------------------------------------------------------------
# Boundary sets
# ----------------------------------------------------------------------------

_FACES = [(0, 0.0, -1.0), (0, 1.0, 1.0), (1, 0.0, -1.0), (1, 1.0, 1.0), (2, 0.0, -1.0), (2, 1.0, 1.0)]


def boundary_nodes(coords):
    on = np.zeros(coords.shape[0], dtype=bool)
    for d, val, _ in _FACES:
        on |= np.isclose(coords[:, d], val)
    return np.nonzero(on)[0].astype(np.int32)


def inflow_nodes(coords, bfield):
    """Nodes on a cube face f with b(x_i) . n_f < 0 (b . n = 0 is not inflow)."""
    bx = eval_field(bfield, coords)
    on = np.zeros(coords.shape[0], dtype=bool)
    for d, val, sgn in _FACES:
        on |= np.isclose(coords[:, d], val) & (sgn * bx[:, d] < 0.0)
    return np.nonzero(on)[0].astype(np.int32)


def faces_nodes(coords, faces):
    """Nodes on the listed faces, e.g. faces = [('x', 0), ('y', 1)]."""
    on = np.zeros(coords.shape[0], dtype=bool)
    for axis, val in faces:
        d = "xyz".index(axis)
        on |= np.isclose(coords[:, d], float(val))
    return np.nonzero(on)[0].astype(np.int32)


# ----------------------------------------------------------------------------
# Generic builder
# ----------------------------------------------------------------------------


def build(elem: str, n: int, eps: float, bfield, c: float, *, load=None, dirichlet="all",
          dir_fn=None, u0_fn=None, params=None) -> Instance:
    """Assemble one instance.

    load: None (F = 0), ('box', lo3, hi3) for the indicator of an axis-aligned
    box (exact for Q1, interpolated for P1), or ('fn', f) for F = M_C f(x_nodes)
    (the interpolated source).  dirichlet: 'all' | 'inflow' | 'none' | list of
    faces | index array.  dir_fn(X) gives u_D (default 0).  u0_fn(X) gives u0.
    """
    if isinstance(bfield, (list, tuple)) and len(bfield) == 3 and np.isscalar(bfield[0]):
        bfield = affine_field(bfield)
    coords = grid_coords(n)
    N = coords.shape[0]
    if elem == "Q1":
        row_ptr, col, valid, ijk = _q1_pattern(n)
        Mt, Et, Ct = _q1_operator_terms(n, eps, bfield, c)
        M = _q1_values(n, valid, ijk, Mt)
        E = _q1_values(n, valid, ijk, Et) if Et else np.zeros_like(M)
        C = _q1_values(n, valid, ijk, Ct) if Ct else np.zeros_like(M)
        del valid
    elif elem == "P1":
        row_ptr, col, M, E, C = _p1_assemble(n, eps, bfield, c)
    else:
        raise ValueError(elem)
    A = E + C
    K = -A
    K_conv = -C
    F = np.zeros(N)
    if load is not None:
        kind = load[0]
        if kind == "box" and elem == "Q1":
            lo, hi = load[1], load[2]
            fx, fy, fz = (_box_load_1d(n, lo[d], hi[d]) for d in range(3))
            F = (fz[:, None, None] * fy[None, :, None] * fx[None, None, :]).ravel()
        elif kind == "box":
            lo, hi = np.asarray(load[1]), np.asarray(load[2])
            fn = ((coords >= lo - 1e-12) & (coords <= hi + 1e-12)).all(axis=1).astype(np.float64)
            F = _csr_matvec(row_ptr, col, M, fn)
        elif kind == "fn":
            F = _csr_matvec(row_ptr, col, M, np.asarray(load[1](coords), dtype=np.float64))
        else:
            raise ValueError(load)
    if isinstance(dirichlet, str):
        if dirichlet == "all":
            dir_idx = boundary_nodes(coords)
        elif dirichlet == "inflow":
            dir_idx = inflow_nodes(coords, bfield)
        elif dirichlet == "none":
            dir_idx = np.zeros(0, dtype=np.int32)
        else:
            raise ValueError(dirichlet)
    elif len(dirichlet) and isinstance(dirichlet[0], tuple):
        dir_idx = faces_nodes(coords, dirichlet)
    else:
        dir_idx = np.asarray(dirichlet, dtype=np.int32)
    dir_idx = np.sort(dir_idx).astype(np.int32)
    dir_val = np.zeros(dir_idx.shape[0]) if dir_fn is None else np.asarray(dir_fn(coords[dir_idx]), dtype=np.float64)
    u0 = np.zeros(N) if u0_fn is None else np.asarray(u0_fn(coords), dtype=np.float64)
    u0 = u0.copy()
    u0[dir_idx] = dir_val
    p = dict(eps=eps, c=c, b0=bfield[0].tolist(), B=bfield[1].tolist())
    if params:
        p.update(params)
    return Instance(elem, n, N, row_ptr, col, M, K, K_conv, F, dir_idx, dir_val, u0, coords, p)


def _csr_matvec(row_ptr, col, val, x):
    rows = np.repeat(np.arange(row_ptr.shape[0] - 1), np.diff(row_ptr))
    return np.bincount(rows, weights=val * x[col], minlength=row_ptr.shape[0] - 1)


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------

CFG1_B = (1.0, -0.5, 0.25)


def _box_indicator(lo, hi):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return lambda X: ((X >= lo - 1e-12) & (X <= hi + 1e-12)).all(axis=1).astype(np.float64)


def config1(n: int = 8) -> Instance:
    """CN-FCT on P1 Kuhn tets: eps=1e-6, b=(1,-0.5,0.25), c=0, f=0,
    u0 = 1 on [0.2,0.45]^3, u = 0 on inflow nodes, dt = 1e-3, 50 steps."""
    return build("P1", n, 1e-6, affine_field(CFG1_B), 0.0, load=None, dirichlet="inflow",
                 u0_fn=_box_indicator([0.2] * 3, [0.45] * 3),
                 params=dict(cfg=1, dt=1e-3, steps=50, lin_atol=1e-12, fp_tol=1e-12, fp_maxit=50, prelimit=2.0))


def config2(n: int = 64) -> Instance:
    """SSP-RK3 + Zalesak FCT on Q1: eps=1e-8, rotating b, seeded ball r=0.15,
    inflow Dirichlet u=0, dt = 0.2 h / max |b(x_i)|, 200 steps."""
    rng = np.random.default_rng((0, 2, 0))
    centre = rng.uniform(0.2, 0.8, size=3)
    bfield = ROTATING_B

    def u0_fn(X):
        return (np.linalg.norm(X - centre[None, :], axis=1) <= 0.15).astype(np.float64)

    inst = build("Q1", n, 1e-8, bfield, 0.0, load=None, dirichlet="inflow", u0_fn=u0_fn)
    bmax = float(np.max(np.linalg.norm(eval_field(bfield, inst.coords), axis=1)))
    dt = 0.2 * (1.0 / n) / bmax
    inst.params.update(cfg=2, dt=dt, steps=200, centre=centre.tolist())
    return inst


def config3(n: int = 128) -> Instance:
    """Stationary MCL on Q1: eps=1e-6, b=(1,1,1)/sqrt(3), c=1,
    f = 1 on [0.25,0.5]^3, u = 0 on the whole boundary."""
    s = 1.0 / math.sqrt(3.0)
    return build("Q1", n, 1e-6, affine_field([s, s, s]), 1.0, load=("box", [0.25] * 3, [0.5] * 3),
                 dirichlet="all", params=dict(cfg=3, fp_rtol=1e-8, lin_rtol=1e-10))


def config4_params(count: int = 256, nmin: int = 8, nmax: int = 32):
    """Seeded coefficients of the batched CN-FCT instances."""
    out = []
    for k in range(count):
        rng = np.random.default_rng((0, 4, k))
        n = int(rng.integers(nmin, nmax + 1))
        eps = float(10.0 ** rng.uniform(-8.0, -3.0))
        g = rng.standard_normal(3)
        b = g / np.linalg.norm(g)
        c = float(rng.uniform(0.0, 1.0))
        out.append(dict(n=n, eps=eps, b=b.tolist(), c=c))
    return out


def config4_instance(p) -> Instance:
    return build("P1", p["n"], p["eps"], affine_field(p["b"]), p["c"], load=None, dirichlet="inflow",
                 u0_fn=_box_indicator([0.2] * 3, [0.45] * 3),
                 params=dict(cfg=4, dt=1e-3, steps=20, lin_atol=1e-12, fp_tol=1e-12, fp_maxit=50, prelimit=2.0))


def manufactured(elem: str, n: int, t: float | None = None):
    """Smooth manufactured solution u* = exp(0.5x + y + 1.5z)/e^3 (times e^-t when
    t is given) for eps = 0.1, b = (1, 0.5, 0.25), c = 1; returns
    (instance with Dirichlet data u* on the whole boundary, exact nodal u*)."""
    eps, b, c = 0.1, np.array([1.0, 0.5, 0.25]), 1.0
    g = np.array([0.5, 1.0, 1.5])
    tf = 1.0 if t is None else math.exp(-t)

    def u_star(X):
        return np.exp(X @ g) / math.e ** 3 * tf

    def f(X):
        u = u_star(X)
        lap = float(g @ g) * u
        adv = float(b @ g) * u
        dudt = -u if t is not None else 0.0
        return dudt - eps * lap + adv + c * u

    inst = build(elem, n, eps, affine_field(b), c, load=("fn", f), dirichlet="all",
                 dir_fn=u_star, u0_fn=u_star)
    return inst, u_star(inst.coords)


def config5_requests(count: int, rate: float = 200.0, nmin: int = 16, nmax: int = 96, seed=(0, 5)):
    """Seeded request stream of the serving workload: exponential inter-arrival
    gaps of mean 1/rate seconds, kind ~ Bernoulli(1/2) between 'cn' (20 CN-FCT
    steps, dt = 1e-3, u0 = 1 on [0.2,0.45]^3, inflow Dirichlet u = 0) and
    'mcl' (stationary, f = 1 on [0.25,0.5]^3, u = 0 on the boundary), Q1 mesh
    n = round(exp(U(ln nmin, ln nmax))), eps = 10^U(-8,-3), |b| = 1 in a
    random direction, c ~ U(0, 1)."""
    rng = np.random.default_rng((*seed, 1))
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for k in range(count):
        r = np.random.default_rng((*seed, 2, k))
        kind = "cn" if r.uniform() < 0.5 else "mcl"
        n = int(round(math.exp(r.uniform(math.log(nmin), math.log(nmax)))))
        eps = float(10.0 ** r.uniform(-8.0, -3.0))
        g = r.standard_normal(3)
        b = (g / np.linalg.norm(g)).tolist()
        c = float(r.uniform(0.0, 1.0))
        out.append(dict(arrival=float(t[k]), kind=kind, n=n, eps=eps, b=b, c=c))
    return out


def config5_instance(req) -> Instance:
    if req["kind"] == "cn":
        return build("Q1", req["n"], req["eps"], affine_field(req["b"]), req["c"], load=None, dirichlet="inflow",
                     u0_fn=_box_indicator([0.2] * 3, [0.45] * 3), params=dict(cfg=5, dt=1e-3, steps=20))
    return build("Q1", req["n"], req["eps"], affine_field(req["b"]), req["c"], load=("box", [0.25] * 3, [0.5] * 3),
                 dirichlet="all", params=dict(cfg=5, fp_rtol=1e-8))


def renumbered(inst: Instance, seed=(0, 9)) -> Instance:
    """The same problem with its nodes renamed by a seeded random permutation
    (node i becomes perm[i]; every CSR row re-sorted by column).  Stands in for
    the unstructured node numbering of a general mesh: neighbouring rows no
    longer share one column-offset pattern."""
    perm = np.random.default_rng(seed).permutation(inst.N)
    rows = inst.row_index()
    new_r = perm[rows]
    new_c = perm[inst.col.astype(np.int64)]
    order = np.lexsort((new_c, new_r))
    counts = np.bincount(new_r, minlength=inst.N)
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)

    def nodal(v):
        out = np.empty_like(v)
        out[perm] = v
        return out

    d_new = perm[inst.dir_idx.astype(np.int64)]
    d_order = np.argsort(d_new)
    return Instance(elem=inst.elem, n=inst.n, N=inst.N, row_ptr=row_ptr, col=new_c[order].astype(np.int32),
                    M=inst.M[order], K=inst.K[order], K_conv=inst.K_conv[order], F=nodal(inst.F),
                    dir_idx=d_new[d_order].astype(np.int32), dir_val=inst.dir_val[d_order], u0=nodal(inst.u0),
                    coords=nodal(inst.coords), params=dict(inst.params, perm=perm))


def with_long_row(inst: Instance, extra: int = 40, seed=(0, 11)) -> Instance:
    """The same problem with its middle node coupled to `extra` further nodes,
    a row longer than any mesh stencil.  The new entries are structurally
    symmetric, carry zero mass and small antisymmetric convective values
    (k_ij = -k_ji in K and K_conv), and the diagonals absorb them so that every
    row of K and K_conv keeps its sum."""
    rng = np.random.default_rng(seed)
    N = inst.N
    node = N // 2
    rows = inst.row_index()
    cols = inst.col.astype(np.int64)
    near = set(cols[inst.row_ptr[node]:inst.row_ptr[node + 1]].tolist())
    cand = np.array([j for j in range(N) if j not in near], dtype=np.int64)
    js = np.sort(rng.choice(cand, size=extra, replace=False))
    a = rng.uniform(-0.01, 0.01, size=extra)
    r_all = np.concatenate([rows, np.full(extra, node), js])
    c_all = np.concatenate([cols, js, np.full(extra, node)])
    order = np.lexsort((c_all, r_all))
    counts = np.bincount(r_all, minlength=N)
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    col = c_all[order].astype(np.int32)

    def coupled(v):
        out = np.concatenate([v, a, -a])[order]
        # diagonal entries absorb the new couplings (row sums unchanged)
        diag = np.empty(N, dtype=np.int64)
        for i in range(N):
            k = row_ptr[i] + np.searchsorted(col[row_ptr[i]:row_ptr[i + 1]], i)
            diag[i] = k
        out[diag[node]] -= a.sum()
        np.add.at(out, diag[js], a)
        return out

    return Instance(elem=inst.elem, n=inst.n, N=N, row_ptr=row_ptr, col=col,
                    M=np.concatenate([inst.M, np.zeros(2 * extra)])[order], K=coupled(inst.K),
                    K_conv=coupled(inst.K_conv), F=inst.F.copy(), dir_idx=inst.dir_idx.copy(),
                    dir_val=inst.dir_val.copy(), u0=inst.u0.copy(), coords=inst.coords.copy(),
                    params=dict(inst.params, long_row=node))


# ----------------------------------------------------------------------------
# The paper's analytic accuracy examples, on this package's meshes
# ----------------------------------------------------------------------------


def rotating_shapes_u0(X):
    """Indicator of the three bodies of the rotating-shapes example: a cube
    (edge 0.25, centre (0.5, 0.25, 0.5)), a cone (height 0.5, base radius
    0.125, base centre (0.75, 0.5, 0.25)) and a hollow cylinder (radii 0.0625
    and 0.125, height 0.5, base centre (0.5, 0.75, 0.25))."""
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    cube = (np.abs(x - 0.5) <= 0.125) & (np.abs(y - 0.25) <= 0.125) & (np.abs(z - 0.5) <= 0.125)
    zc = z - 0.25
    tall = (zc >= 0.0) & (zc <= 0.5)
    cone = tall & (np.hypot(x - 0.75, y - 0.5) <= 0.125 * (1.0 - zc / 0.5))
    rh = np.hypot(x - 0.5, y - 0.75)
    hollow = tall & (rh >= 0.0625) & (rh <= 0.125)
    return (cube | cone | hollow).astype(np.float64)


def rotating_shapes(n: int = 64) -> Instance:
    """Rotating bodies (the paper's first time-dependent example): eps = 0,
    b = (0.5 - y, x - 0.5, 0), c = 0, f = 0, u = 0 on the whole boundary, one
    full rotation T = 2 pi.  Q1 on n^3 cubes; dt = 1e-3 * 256 / n keeps the
    paper's ratio dt / h (h = 2^-8, dt = 1e-3)."""
    dt = 1e-3 * 256.0 / n
    steps = int(round(2.0 * math.pi / dt))
    b = affine_field([0.5, -0.5, 0.0], [[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    return build("Q1", n, 0.0, b, 0.0, dirichlet="all", u0_fn=rotating_shapes_u0,
                 params=dict(example="rotating_shapes", dt=dt, steps=steps, T=steps * dt))


def circular_convection_exact(X):
    """Exact solution of the circular-convection example, r = sqrt(x^2 + y^2):
    1 on 0.15 <= r <= 0.45, cos^2(10 pi (r - 0.7) / 3) on 0.55 <= r <= 0.85,
    0 elsewhere."""
    r = np.hypot(X[:, 0], X[:, 1])
    u = np.zeros(X.shape[0])
    u[(r >= 0.15) & (r <= 0.45)] = 1.0
    m = (r >= 0.55) & (r <= 0.85)
    u[m] = np.cos(10.0 * math.pi * (r[m] - 0.7) / 3.0) ** 2
    return u


def circular_convection(n: int = 32, elem: str = "P1") -> Instance:
    """Circular convection (the paper's stationary accuracy example): eps = 0,
    b = (y, -x, 0), c = 0, f = 0, Dirichlet data from the exact solution on
    the faces y = 1, x = 0 and x = 1, natural conditions elsewhere."""
    b = affine_field([0.0, 0.0, 0.0], [[0.0, 1.0, 0.0], [-1.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    return build(elem, n, 0.0, b, 0.0, dirichlet=[("y", 1), ("x", 0), ("x", 1)], dir_fn=circular_convection_exact,
                 params=dict(example="circular_convection"))
