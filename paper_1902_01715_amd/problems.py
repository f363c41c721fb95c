"""Seeded synthetic linear-elasticity problems K u = f (the solver's inputs).

This module only *generates inputs*: structured trilinear hexahedral (Q1) meshes,
the stiffness matrix K = sum_e int B^T D B dV (the paper's problem statement,
Section 1, eq. (1) and the text that follows it), consistent loads, clamped
boundary conditions and the six rigid-body modes used as the initial test space
(Section 3.3).  It contains none of the AMG method's arithmetic, and both the
GPU path and the CPU oracle read the arrays it returns.

Conventions
-----------
* node id   = i + (nx+1) * (j + (ny+1) * k)
* element id = i + nx * (j + ny * k)
* local node order of a hexahedron: 0 (-,-,-), 1 (+,-,-), 2 (+,+,-), 3 (-,+,-),
  then 4..7 the same at +zeta.
* DOF index = 3 * node + component.
* Element: 2x2x2 Gauss-Legendre, isotropic D in Voigt order
  (xx, yy, zz, yz, xz, xy) with engineering shears.
* Clamped nodes: all three DOFs fixed.  Their rows and columns are removed
  symmetrically: the diagonal block becomes I3, every coupling block to or from
  a clamped node is dropped from the pattern, and f = 0 there.
* K is returned as 3x3-block CSR (BSR): row_ptr int32 [N+1], col int32 [nnzb]
  sorted ascending per row, vals float64 [nnzb, 3, 3] row-major blocks.
* Random draws use numpy.random.default_rng(seed) (PCG64) in a fixed order.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

_SIGNS = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                   [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)
_LOCAL_OFF = ((_SIGNS + 1) // 2).astype(np.int64)   # (8,3) 0/1 offsets of local nodes
_GP = 1.0 / math.sqrt(3.0)


@dataclasses.dataclass
class Problem:
    """A synthetic elasticity system in the solver's input layout."""
    name: str
    shape: tuple            # (nx, ny, nz) elements
    coords: np.ndarray      # (N, 3) float64
    conn: np.ndarray        # (n_el, 8) int32
    row_ptr: np.ndarray     # (N+1,) int32
    col: np.ndarray         # (nnzb,) int32
    vals: np.ndarray        # (nnzb, 3, 3) float64
    f: np.ndarray           # (N*3,) float64 or (N*3, k) for several load cases
    V0: np.ndarray          # (N, 3, 6) rigid-body modes, node-major
    dirichlet: np.ndarray   # (N,) bool
    E: np.ndarray           # (n_el,) Young's modulus per element
    nu: np.ndarray          # (n_el,) Poisson ratio per element
    Ke0: np.ndarray | None = None   # (24,24) shared unit-modulus element matrix, if uniform
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return self.coords.shape[0]

    @property
    def n_dof(self) -> int:
        return 3 * self.coords.shape[0]

    @property
    def nnzb(self) -> int:
        return int(self.col.shape[0])

    def to_scipy(self):
        """K as a scipy.sparse BSR matrix (for tests)."""
        import scipy.sparse as sp
        N = self.n_nodes
        return sp.bsr_matrix((self.vals, self.col, self.row_ptr), shape=(3 * N, 3 * N))


# ----------------------------------------------------------------------------
# mesh
# ----------------------------------------------------------------------------
def structured_nodes(nx, ny, nz, lx, ly, lz):
    i = np.arange(nx + 1, dtype=np.float64) * (lx / nx)
    j = np.arange(ny + 1, dtype=np.float64) * (ly / ny)
    k = np.arange(nz + 1, dtype=np.float64) * (lz / nz)
    Z, Y, X = np.meshgrid(k, j, i, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def structured_conn(nx, ny, nz):
    ei, ej, ek = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    # element id = i + nx*(j + ny*k): iterate k slowest
    ei = ei.transpose(2, 1, 0).ravel()
    ej = ej.transpose(2, 1, 0).ravel()
    ek = ek.transpose(2, 1, 0).ravel()
    nxp, nyp = nx + 1, ny + 1
    conn = np.empty((ei.size, 8), dtype=np.int64)
    for a in range(8):
        oi, oj, ok = _LOCAL_OFF[a]
        conn[:, a] = (ei + oi) + nxp * ((ej + oj) + nyp * (ek + ok))
    return conn


def boundary_node_mask(nx, ny, nz):
    i = np.arange(nx + 1)
    j = np.arange(ny + 1)
    k = np.arange(nz + 1)
    K, J, I = np.meshgrid(k, j, i, indexing="ij")
    b = (I == 0) | (I == nx) | (J == 0) | (J == ny) | (K == 0) | (K == nz)
    return b.ravel()


# ----------------------------------------------------------------------------
# element matrices
# ----------------------------------------------------------------------------
def _dN_dxi():
    """(8 gauss points, 8 nodes, 3) derivatives of the Q1 shape functions."""
    gps = _SIGNS * _GP                     # gauss points in the same sign order
    d = np.empty((8, 8, 3))
    for g in range(8):
        xi = gps[g]
        for a in range(8):
            s = _SIGNS[a]
            f = 1.0 + s * xi
            d[g, a, 0] = 0.125 * s[0] * f[1] * f[2]
            d[g, a, 1] = 0.125 * s[1] * f[0] * f[2]
            d[g, a, 2] = 0.125 * s[2] * f[0] * f[1]
    return d


def _N_at_gp():
    gps = _SIGNS * _GP
    N = np.empty((8, 8))
    for g in range(8):
        N[g] = 0.125 * np.prod(1.0 + _SIGNS * gps[g], axis=1)
    return N


_DNDXI = _dN_dxi()
_NGP = _N_at_gp()


def _bmat(X):
    """B matrices and det J for elements with node coordinates X (ne, 8, 3).

    Returns B (ne, 8gp, 6, 24) and detJ (ne, 8gp)."""
    J = np.einsum("gaj,eai->egij", _DNDXI, X)          # J[i][j] = dx_i/dxi_j
    detJ = np.linalg.det(J)
    if np.any(detJ <= 0):
        raise ValueError("non-positive Jacobian determinant in mesh")
    Jinv = np.linalg.inv(J)                              # Jinv[j][i] = dxi_j/dx_i
    dNdx = np.einsum("gaj,egji->egai", _DNDXI, Jinv)     # (ne, g, a, i)
    ne = X.shape[0]
    B = np.zeros((ne, 8, 6, 24))
    Nx, Ny, Nz = dNdx[..., 0], dNdx[..., 1], dNdx[..., 2]
    B[:, :, 0, 0::3] = Nx
    B[:, :, 1, 1::3] = Ny
    B[:, :, 2, 2::3] = Nz
    B[:, :, 3, 1::3] = Nz
    B[:, :, 3, 2::3] = Ny
    B[:, :, 4, 0::3] = Nz
    B[:, :, 4, 2::3] = Nx
    B[:, :, 5, 0::3] = Ny
    B[:, :, 5, 1::3] = Nx
    return B, detJ


def lame(E, nu):
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def element_stiffness(X, lam, mu):
    """K_e = sum_gp B^T D B detJ for elements X (ne,8,3) with Lame parameters."""
    X = np.asarray(X, dtype=np.float64)
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), (X.shape[0],))
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), (X.shape[0],))
    B, detJ = _bmat(X)
    DB = np.empty_like(B)
    tr = B[:, :, 0] + B[:, :, 1] + B[:, :, 2]
    for r in range(3):
        DB[:, :, r] = lam[:, None, None] * tr + 2.0 * mu[:, None, None] * B[:, :, r]
    for r in range(3, 6):
        DB[:, :, r] = mu[:, None, None] * B[:, :, r]
    DB *= detJ[:, :, None, None]
    ne = X.shape[0]
    Bt = B.transpose(0, 3, 1, 2).reshape(ne, 24, 48)
    DBs = DB.reshape(ne, 48, 24)
    return np.matmul(Bt, DBs)


def unit_element_parts(X1):
    """(K_lambda, K_mu) of one element geometry X1 (8,3): K_e = lam*K_l + mu*K_m."""
    Kl = element_stiffness(X1[None], 1.0, 0.0)[0]
    Km = element_stiffness(X1[None], 0.0, 1.0)[0]
    return Kl, Km


# ----------------------------------------------------------------------------
# BSR pattern and assembly
# ----------------------------------------------------------------------------
_OFFS = np.array([(di, dj, dk) for dk in (-1, 0, 1) for dj in (-1, 0, 1) for di in (-1, 0, 1)],
                 dtype=np.int64)   # ordered so that neighbour ids ascend


def structured_pattern(nx, ny, nz, dirichlet):
    """27-point node pattern with clamped couplings removed.

    Returns row_ptr, col (int32) and slot27 (N, 27) int64 giving the position of
    each (node, offset) block in col, or -1 if absent."""
    nxp, nyp, nzp = nx + 1, ny + 1, nz + 1
    N = nxp * nyp * nzp
    ids = np.arange(N, dtype=np.int64)
    I = ids % nxp
    J = (ids // nxp) % nyp
    K = ids // (nxp * nyp)
    valid = np.zeros((N, 27), dtype=bool)
    nb = np.full((N, 27), -1, dtype=np.int64)
    for o, (di, dj, dk) in enumerate(_OFFS):
        ii, jj, kk = I + di, J + dj, K + dk
        ok = (ii >= 0) & (ii < nxp) & (jj >= 0) & (jj < nyp) & (kk >= 0) & (kk < nzp)
        nid = ii + nxp * (jj + nyp * kk)
        center = (di == 0 and dj == 0 and dk == 0)
        if not center:
            ok &= ~dirichlet
            ok &= ~dirichlet[np.where(ok, nid, 0)]
        valid[:, o] = ok
        nb[:, o] = np.where(ok, nid, -1)
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    pos = np.cumsum(valid, axis=1) - 1 + row_ptr[:-1, None]
    slot27 = np.where(valid, pos, -1)
    col = nb[valid]
    if row_ptr[-1] >= 2**31:
        raise ValueError("pattern too large for int32 indices")
    return row_ptr.astype(np.int32), col.astype(np.int32), slot27


def assemble(nx, ny, nz, conn, dirichlet, row_ptr, slot27, ke_fn, chunk=65536):
    """Scatter element matrices into BSR values.

    ke_fn(e0, e1) returns the (e1-e0, 24, 24) element matrices of elements e0..e1-1.
    For a fixed pair of local nodes (a, b) every element maps to a distinct
    block, so each of the 64 (a, b) passes is a plain vectorised add."""
    nnzb = int(row_ptr[-1])
    vals = np.zeros((nnzb, 3, 3))
    n_el = conn.shape[0]
    nxp, nyp = nx + 1, ny + 1
    # offset index (0..26) of node b relative to node a
    off_idx = np.empty((8, 8), dtype=np.int64)
    for a in range(8):
        for b in range(8):
            d = _LOCAL_OFF[b] - _LOCAL_OFF[a]
            off_idx[a, b] = (d[0] + 1) + 3 * (d[1] + 1) + 9 * (d[2] + 1)
    for e0 in range(0, n_el, chunk):
        e1 = min(n_el, e0 + chunk)
        Ke = ke_fn(e0, e1).reshape(e1 - e0, 8, 3, 8, 3)
        for a in range(8):
            rows = conn[e0:e1, a]
            for b in range(8):
                slots = slot27[rows, off_idx[a, b]]
                m = slots >= 0
                if not m.any():
                    continue
                vals[slots[m]] += Ke[m, a, :, b, :]
    # make K bitwise symmetric: block (r, c) and block (c, r)^T are averaged; the
    # mirror of offset o is offset 26 - o in the neighbour's row.
    N = slot27.shape[0]
    node = np.repeat(np.arange(N), 27).reshape(N, 27)
    ids = np.arange(N, dtype=np.int64)
    nxq = nx + 1
    nyq = ny + 1
    for o, (di, dj, dk) in enumerate(_OFFS):
        if o >= 13:
            break
        s = slot27[:, o]
        m = s >= 0
        r = ids[m]
        c = r + di + nxq * (dj + nyq * dk)
        t = slot27[c, 26 - o]
        a = vals[s[m]]
        bT = vals[t].transpose(0, 2, 1)
        avg = (a + bT) * 0.5
        vals[s[m]] = avg
        vals[t] = avg.transpose(0, 2, 1)
    dg = slot27[:, 13]
    vals[dg] = (vals[dg] + vals[dg].transpose(0, 2, 1)) * 0.5
    # clamped diagonal blocks := I3
    dn = np.nonzero(dirichlet)[0]
    if dn.size:
        diag = slot27[dn, 13]
        vals[diag] = np.eye(3)
    return vals


def rigid_body_modes(coords):
    """Six rigid-body modes (3 translations, 3 rotations about the centroid), node-major."""
    N = coords.shape[0]
    c = coords - coords.mean(axis=0)
    V = np.zeros((N, 3, 6))
    V[:, 0, 0] = 1.0
    V[:, 1, 1] = 1.0
    V[:, 2, 2] = 1.0
    # rotation about x: e_x cross r = (0, -r_z, r_y)
    V[:, 1, 3] = -c[:, 2]
    V[:, 2, 3] = c[:, 1]
    # about y: (r_z, 0, -r_x)
    V[:, 0, 4] = c[:, 2]
    V[:, 2, 4] = -c[:, 0]
    # about z: (-r_y, r_x, 0)
    V[:, 0, 5] = -c[:, 1]
    V[:, 1, 5] = c[:, 0]
    return V


def initial_test_space(p, n_tv, seed):
    """Initial test space [N, b, n_tv]: the near-null space of p (the six
    rigid-body modes, or the constant of a scalar problem), then columns of
    seeded standard normal entries up to n_tv (the random padding of the test
    space is an input)."""
    k = p.V0.shape[2]
    if n_tv < k:
        raise ValueError(f"n_tv must be at least {k}")
    extra = np.random.default_rng(seed).standard_normal((p.V0.shape[0], p.V0.shape[1], n_tv - k))
    return np.ascontiguousarray(np.concatenate([p.V0, extra], axis=2))


def body_force(coords, conn, b, chunk=65536):
    """Consistent nodal loads of a uniform body force b (per unit volume)."""
    N = coords.shape[0]
    f = np.zeros((N, 3))
    b = np.asarray(b, dtype=np.float64)
    for e0 in range(0, conn.shape[0], chunk):
        e1 = min(conn.shape[0], e0 + chunk)
        X = coords[conn[e0:e1]]
        J = np.einsum("gaj,eai->egij", _DNDXI, X)
        detJ = np.linalg.det(J)
        w = np.einsum("ga,eg->ea", _NGP, detJ)             # int N_a dV
        for a in range(8):
            np.add.at(f, conn[e0:e1, a], w[:, a, None] * b[None, :])
    return f


def face_traction(coords, conn, face_elems, face_local, t):
    """Consistent nodal loads of a uniform traction t on a planar axis-aligned face.

    face_elems: element ids on the face; face_local: the 4 local node ids of the face.
    Each bilinear face node receives t * area / 4 (exact for rectangular faces)."""
    N = coords.shape[0]
    f = np.zeros((N, 3))
    t = np.asarray(t, dtype=np.float64)
    nodes = conn[face_elems][:, face_local]               # (nf, 4)
    P = coords[nodes]
    area = np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 3] - P[:, 0]), axis=1)
    for a in range(4):
        np.add.at(f, nodes[:, a], (area / 4.0)[:, None] * t[None, :])
    return f


# ----------------------------------------------------------------------------
# generic structured box problem
# ----------------------------------------------------------------------------
def box_problem(name, nx, ny, nz, lx, ly, lz, *, E, nu, clamp="z0", load=("body", (0, 0, -1)),
                jitter=0.0, rng=None, scaled_uniform=False):
    """Assemble a structured box.

    E, nu: scalars or per-element arrays.  clamp: 'z0' or 'x0' or None.
    load: ('body', b) | ('traction', face, t) | ('none',).
    jitter: interior nodes moved by U[-jitter*h, jitter*h] per coordinate (h per axis).
    scaled_uniform: if True (uniform geometry and nu), K_e = E_e * Ke0 exactly."""
    coords = structured_nodes(nx, ny, nz, lx, ly, lz)
    N = coords.shape[0]
    if jitter > 0.0:
        d = rng.uniform(-1.0, 1.0, size=(N, 3))
        h = np.array([lx / nx, ly / ny, lz / nz])
        interior = ~boundary_node_mask(nx, ny, nz)
        coords[interior] += jitter * d[interior] * h[None, :]
    conn = structured_conn(nx, ny, nz)
    n_el = conn.shape[0]
    E = np.broadcast_to(np.asarray(E, dtype=np.float64), (n_el,)).copy()
    nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), (n_el,)).copy()

    ids = np.arange(N)
    I = ids % (nx + 1)
    K = ids // ((nx + 1) * (ny + 1))
    if clamp == "z0":
        dirichlet = K == 0
    elif clamp == "x0":
        dirichlet = I == 0
    elif clamp is None:
        dirichlet = np.zeros(N, dtype=bool)
    else:
        raise ValueError(clamp)

    row_ptr, col, slot27 = structured_pattern(nx, ny, nz, dirichlet)
    Ke0 = None
    if jitter == 0.0:
        X1 = coords[conn[0]]
        Kl, Km = unit_element_parts(X1)
        if scaled_uniform:
            l0, m0 = lame(1.0, nu[0])
            Ke0 = l0 * Kl + m0 * Km
            Ke0 = (Ke0 + Ke0.T) * 0.5
            ke_fn = lambda e0, e1: E[e0:e1, None, None] * Ke0[None]
        else:
            lam, mu = lame(E, nu)
            ke_fn = lambda e0, e1: lam[e0:e1, None, None] * Kl[None] + mu[e0:e1, None, None] * Km[None]
    else:
        lam, mu = lame(E, nu)
        ke_fn = lambda e0, e1: element_stiffness(coords[conn[e0:e1]], lam[e0:e1], mu[e0:e1])
    vals = assemble(nx, ny, nz, conn, dirichlet, row_ptr, slot27, ke_fn)

    if load[0] == "body":
        f = body_force(coords, conn, load[1])
    elif load[0] == "traction":
        face, t = load[1], load[2]
        eid = np.arange(n_el)
        ei = eid % nx
        ek = eid // (nx * ny)
        if face == "x1":
            fe = eid[ei == nx - 1]
            fl = [1, 2, 6, 5]
        elif face == "z1":
            fe = eid[ek == nz - 1]
            fl = [4, 5, 6, 7]
        else:
            raise ValueError(face)
        f = face_traction(coords, conn, fe, fl, t)
    elif load[0] == "none":
        f = np.zeros((N, 3))
    else:
        raise ValueError(load)
    f[dirichlet] = 0.0
    V0 = rigid_body_modes(coords)
    return Problem(name=name, shape=(nx, ny, nz), coords=coords, conn=conn.astype(np.int32),
                   row_ptr=row_ptr, col=col, vals=vals, f=f.reshape(-1), V0=V0,
                   dirichlet=dirichlet, E=E, nu=nu, Ke0=Ke0)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
def c1_cube(n=10):
    """Unit cube, n^3 Q1 hexes, E=1, nu=0.3, z=0 clamped, body force (0,0,-1)."""
    return box_problem(f"cube{n}", n, n, n, 1.0, 1.0, 1.0, E=1.0, nu=0.3, clamp="z0",
                       load=("body", (0.0, 0.0, -1.0)), scaled_uniform=True)


def c2_cantilever(nx=320, ny=32, nz=32, seed=2):
    """Cantilever [0,100]x[0,1]x[0,1], aspect-10 elements, log-uniform E in [1e-3,1e3],
    nu ~ U[0.25,0.45], clamped at x=0, unit traction (0,0,-1) on the x=100 face."""
    rng = np.random.default_rng(seed)
    n_el = nx * ny * nz
    log10E = rng.uniform(-3.0, 3.0, size=n_el)
    nu = rng.uniform(0.25, 0.45, size=n_el)
    E = 10.0 ** log10E
    lx = 100.0 * nx / 320.0
    ly = 1.0 * ny / 32.0
    lz = 1.0 * nz / 32.0
    return box_problem(f"cantilever{nx}x{ny}x{nz}", nx, ny, nz, lx, ly, lz, E=E, nu=nu,
                       clamp="x0", load=("traction", "x1", (0.0, 0.0, -1.0)))


def c3_layered_distorted(nx=128, ny=128, nz=64, seed=3):
    """[0,1]x[0,1]x[0,nz/128] with h = 1/128, interior nodes jittered by U[-0.3h,0.3h],
    E = 1 / 1e4 alternating every 8 element layers in z, nu=0.3, z=0 clamped,
    body force (0,0,-1)."""
    rng = np.random.default_rng(seed)
    n_el = nx * ny * nz
    ek = np.arange(n_el) // (nx * ny)
    E = np.where((ek // 8) % 2 == 0, 1.0, 1.0e4)
    return box_problem(f"layered{nx}x{ny}x{nz}", nx, ny, nz, nx / 128.0, ny / 128.0, nz / 128.0,
                       E=E, nu=0.3, clamp="z0", load=("body", (0.0, 0.0, -1.0)),
                       jitter=0.3, rng=rng)


def c4_multiload(n=96, k=32, seed=4):
    """Unit cube n^3, E=1, nu=0.3, z=0 clamped, k load cases of N(0,1) nodal forces on
    the top-face nodes.  f has shape (3N, k)."""
    p = box_problem(f"cube{n}x{k}rhs", n, n, n, 1.0, 1.0, 1.0, E=1.0, nu=0.3, clamp="z0",
                    load=("none",), scaled_uniform=True)
    rng = np.random.default_rng(seed)
    N = p.n_nodes
    top = np.arange(N)[np.arange(N) // ((n + 1) * (n + 1)) == n]
    F = np.zeros((N, 3, k))
    F[top] = rng.standard_normal((top.size, 3, k))
    p.f = F.reshape(3 * N, k)
    return p


def c5_simp(n=48, seed=5, n_fd=20):
    """Unit cube n^3, SIMP density rho ~ U[0.1,1], E = rho^3, nu = 0.3, z=0 clamped,
    traction (0,0,-1) on z=1.  extra['rho'], extra['fd_elems'] hold the draws."""
    rng = np.random.default_rng(seed)
    n_el = n ** 3
    rho = rng.uniform(0.1, 1.0, size=n_el)
    fd = rng.choice(n_el, size=min(n_fd, n_el), replace=False)
    p = box_problem(f"simp{n}", n, n, n, 1.0, 1.0, 1.0, E=rho ** 3, nu=0.3, clamp="z0",
                    load=("traction", "z1", (0.0, 0.0, -1.0)), scaled_uniform=True)
    p.extra["rho"] = rho
    p.extra["fd_elems"] = fd
    return p


def unconstrained_box(nx, ny, nz, lx=1.0, ly=1.0, lz=1.0, E=1.0, nu=0.3, jitter=0.0, seed=0):
    """Box without boundary conditions (singular K; used for null-space and patch checks)."""
    rng = np.random.default_rng(seed)
    return box_problem(f"free{nx}x{ny}x{nz}", nx, ny, nz, lx, ly, lz, E=E, nu=nu, clamp=None,
                       load=("none",), jitter=jitter, rng=rng)


CONFIGS = {
    "c1": c1_cube,
    "c2": c2_cantilever,
    "c3": c3_layered_distorted,
    "c4": c4_multiload,
    "c5": c5_simp,
}


# ----------------------------------------------------------------------------
# Scalar (point-wise) inputs on linear tetrahedra (P1), the element family of
# most of the paper's test matrices (Section 4, Table "Test matrices"), in
# plain CSR for the block size b = 1.
# ----------------------------------------------------------------------------
# the six tetrahedra of a hexahedron sharing its diagonal 0-6 (local hex node
# numbers as above); neighbouring hexahedra split their shared faces alike
_HEX_TETS = np.array([[0, 1, 2, 6], [0, 2, 3, 6], [0, 3, 7, 6], [0, 7, 4, 6], [0, 4, 5, 6], [0, 5, 1, 6]])


@dataclasses.dataclass
class ScalarProblem:
    """A synthetic SPD system in scalar CSR (block size 1)."""
    name: str
    coords: np.ndarray      # (N, 3) nodes of the mesh
    tets: np.ndarray        # (n_el, 4) int64
    row_ptr: np.ndarray     # (n+1,) int32
    col: np.ndarray         # (nnz,) int32, ascending per row
    vals: np.ndarray        # (nnz, 1, 1) float64
    f: np.ndarray           # (n,) float64
    V0: np.ndarray          # (n, 1, n_tv) near-null space of the operator without constraints
    dirichlet: np.ndarray   # (n,) bool: decoupled unknowns (identity rows)

    @property
    def n(self) -> int:
        return self.row_ptr.size - 1

    @property
    def n_dof(self) -> int:
        return self.n

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals.reshape(-1), self.col, self.row_ptr), shape=(self.n, self.n))


def tet_mesh(nx, ny, nz, jitter=0.2, seed=0):
    """Unit box in nx*ny*nz hexahedra, six tetrahedra each, interior nodes
    moved by U[-jitter h, jitter h] per axis (seeded)."""
    coords = structured_nodes(nx, ny, nz, 1.0, 1.0, 1.0)
    hexes = structured_conn(nx, ny, nz).astype(np.int64)
    if jitter > 0:
        h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
        move = np.random.default_rng(seed).uniform(-jitter, jitter, coords.shape) * h
        inner = ~boundary_node_mask(nx, ny, nz)
        coords = coords + np.where(inner[:, None], move, 0.0)
    tets = hexes[:, _HEX_TETS].reshape(-1, 4)
    # positive orientation
    X = coords[tets]
    vol = np.einsum("ij,ij->i", np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), X[:, 3] - X[:, 0])
    flip = vol < 0
    tets[flip] = tets[flip][:, [0, 2, 1, 3]]
    return coords, tets


def _tet_gradients(X):
    """Gradients of the four P1 shape functions and the volumes of tetrahedra X (n_el, 4, 3)."""
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)   # columns: edges
    vol = np.linalg.det(J) / 6.0
    Jinv = np.linalg.inv(J)                     # rows: gradients of barycentric coordinates 1..3
    g = np.empty((X.shape[0], 4, 3))
    g[:, 1:] = Jinv
    g[:, 0] = -Jinv.sum(axis=1)
    return g, vol


def _csr_with_identity_rows(rows, cols, vals, n, fixed):
    """Assembled CSR with the fixed unknowns decoupled: their rows and
    columns dropped and a unit diagonal in their place."""
    import scipy.sparse as sp
    keep = np.logical_not(fixed[rows])
    keep &= np.logical_not(fixed[cols])
    idx = np.flatnonzero(keep)
    A = sp.coo_matrix((vals[idx], (rows[idx], cols[idx])), shape=(n, n)).tocsr()
    A = A + sp.diags(fixed.astype(np.float64))
    A = A.tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def tet_diffusion(nx, ny, nz, contrast=1e3, layers=4, jitter=0.2, seed=0):
    """-div(kappa grad u) = 1 on P1 tetrahedra, u = 0 on z = 0, kappa = 1 and
    `contrast` in alternating layers along z.  Test space: the constant."""
    coords, tets = tet_mesh(nx, ny, nz, jitter, seed)
    g, vol = _tet_gradients(coords[tets])
    zc = coords[tets][:, :, 2].mean(axis=1)
    kappa = np.where((np.floor(zc * layers) % 2) == 1, contrast, 1.0)
    Ke = (kappa * vol)[:, None, None] * np.einsum("eak,ebk->eab", g, g)
    n = coords.shape[0]
    rows = np.repeat(tets, 4, axis=1).reshape(-1)
    cols = np.tile(tets, (1, 4)).reshape(-1)
    fixed = np.isclose(coords[:, 2], 0.0)
    A = _csr_with_identity_rows(rows, cols, Ke.reshape(-1), n, fixed)
    f = np.zeros(n)
    np.add.at(f, tets.reshape(-1), np.repeat(vol / 4.0, 4))
    f[fixed] = 0.0
    V0 = np.ones((n, 1, 1))
    return ScalarProblem(f"tetdiff{nx}x{ny}x{nz}", coords, tets, A.indptr.astype(np.int32),
                         A.indices.astype(np.int32), A.data.reshape(-1, 1, 1).copy(), f, V0, fixed)


def tet_elasticity(nx, ny, nz, E=1.0, nu=0.3, jitter=0.2, seed=0):
    """Linear elasticity on P1 tetrahedra taken point-wise (one unknown per
    displacement component, DOF = 3 node + component), clamped at z = 0,
    uniform body force (0, 0, -1).  Test space: the six rigid-body modes, one
    row per scalar unknown."""
    coords, tets = tet_mesh(nx, ny, nz, jitter, seed)
    g, vol = _tet_gradients(coords[tets])
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2 * mu
    D[np.arange(3, 6), np.arange(3, 6)] = mu
    n_el = tets.shape[0]
    B = np.zeros((n_el, 6, 12))
    for a in range(4):
        gx, gy, gz = g[:, a, 0], g[:, a, 1], g[:, a, 2]
        B[:, 0, 3 * a] = gx
        B[:, 1, 3 * a + 1] = gy
        B[:, 2, 3 * a + 2] = gz
        B[:, 3, 3 * a + 1], B[:, 3, 3 * a + 2] = gz, gy
        B[:, 4, 3 * a], B[:, 4, 3 * a + 2] = gz, gx
        B[:, 5, 3 * a], B[:, 5, 3 * a + 1] = gy, gx
    Ke = vol[:, None, None] * np.matmul(B.transpose(0, 2, 1), np.matmul(D, B))
    dofs = (3 * tets[:, :, None] + np.arange(3)).reshape(n_el, 12).astype(np.int32)
    n = 3 * coords.shape[0]
    rows = np.repeat(dofs, 12, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, 12)).reshape(-1)
    fixed = np.repeat(np.isclose(coords[:, 2], 0.0), 3)
    A = _csr_with_identity_rows(rows, cols, Ke.reshape(-1), n, fixed)
    f = np.zeros(n)
    np.add.at(f, dofs[:, 2::3].reshape(-1), -np.repeat(vol / 4.0, 4))
    f[fixed] = 0.0
    V0 = rigid_body_modes(coords).reshape(n, 1, 6)
    return ScalarProblem(f"tetelast{nx}x{ny}x{nz}", coords, tets, A.indptr.astype(np.int32),
                         A.indices.astype(np.int32), A.data.reshape(-1, 1, 1).copy(), f, V0, fixed)


def t1_tet_elasticity(n=64, seed=6):
    """Point-wise elasticity on n^3 x 6 P1 tetrahedra (3 (n+1)^3 unknowns,
    823,875 for n = 64), interior jitter U[-0.2h, 0.2h], clamped at z = 0,
    body force: the scalar (block size 1) workload."""
    return tet_elasticity(n, n, n, jitter=0.2, seed=seed)


CONFIGS["t1"] = t1_tet_elasticity
