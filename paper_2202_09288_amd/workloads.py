"""Seeded synthetic SPD inputs and their nested-dissection orderings.

This module is the only code shared by the CPU oracle and the HIP library: it
draws random numbers and lays out grid operators, and it holds none of the
factorization's arithmetic.  Every matrix is emitted as the lower triangle
(diagonal included) in compressed-column form with rows sorted ascending:

    colptr  int64[n+1]   column j holds entries colptr[j] .. colptr[j+1]-1
    rowidx  int32[nnz]   row index of each entry, rowidx >= column
    values  float64[nnz]

plus a fill-reducing ordering ``perm`` (int32[n]; perm[k] is the original index
of the k-th pivot).  The paper runs SuiteSparse matrices ordered by METIS or
AMD (Sec. 2, "Background on CHOLMOD"); the grid families below stand in for
them and the ordering is geometric nested dissection from grid coordinates.

Random numbers come from SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), one stream per (workload, seed,
purpose); a double is the top 53 bits times 2^-53.
"""
from __future__ import annotations

import dataclasses
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# purpose tags of the random streams
P_EDGE, P_RHS, P_EIG, P_ROT, P_KIND, P_SIDE, P_POWER, P_ARRIVAL, P_MIX = range(1, 10)


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(workload: int, seed: int, purpose: int, sub: int = 0) -> int:
    """64-bit key of one random stream; distinct tuples give unrelated streams."""
    with np.errstate(over="ignore"):
        k = np.uint64(0)
        for part in (workload, seed, purpose, sub):
            k = _mix(np.array([k + np.uint64(part & 0xFFFFFFFFFFFFFFFF) * _GAMMA + _GAMMA],
                              dtype=np.uint64))[0]
    return int(k)


def splitmix64(key: int, count: int) -> np.ndarray:
    """First ``count`` outputs of SplitMix64 started at state ``key``."""
    with np.errstate(over="ignore"):
        i = np.arange(1, count + 1, dtype=np.uint64)
        return _mix(np.uint64(key) + i * _GAMMA)


def uniform(key: int, count: int) -> np.ndarray:
    """Doubles in [0, 1): top 53 bits of each SplitMix64 output times 2^-53."""
    return (splitmix64(key, count) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# ----------------------------------------------------------------------------
# grids and orderings
# ----------------------------------------------------------------------------

def grid_index(dims):
    """Node id of each grid point, x fastest: id = x + nx*(y + ny*z)."""
    return np.arange(int(np.prod(dims)), dtype=np.int64).reshape(tuple(reversed(dims)))


def nd_perm(dims, dof: int = 1) -> np.ndarray:
    """Geometric nested dissection of a box grid.

    Recursive bisection: split the longest axis (ties go to the lower axis,
    x before y before z) at the plane lo + floor(len/2); order the low half,
    then the high half, then the separator plane, whose points are listed
    lexicographically with x fastest; recurse down to single points.  The dofs
    of a point are consecutive.  Returns perm with perm[k] = original index of
    the k-th pivot.
    """
    dims = tuple(int(d) for d in dims)
    nd = len(dims)
    strides = [1] * nd
    for a in range(1, nd):
        strides[a] = strides[a - 1] * dims[a - 1]
    out = np.empty(int(np.prod(dims)), dtype=np.int64)
    pos = 0

    def emit_box(lo, hi):
        nonlocal pos
        axes = [np.arange(lo[a], hi[a], dtype=np.int64) * strides[a] for a in range(nd)]
        ids = axes[0]
        for a in range(1, nd):  # later axes vary slowest
            ids = (axes[a][:, None] + ids[None, :]).ravel()
        out[pos:pos + ids.size] = ids
        pos += ids.size

    stack = [(tuple(0 for _ in dims), dims, 0)]
    # explicit stack: (lo, hi, state); state 0 = split, 1 = emit separator
    while stack:
        lo, hi, state = stack.pop()
        lens = [hi[a] - lo[a] for a in range(nd)]
        if min(lens) <= 0:
            continue
        if state == 1:
            emit_box(lo, hi)
            continue
        if max(lens) == 1:
            emit_box(lo, hi)
            continue
        axis = max(range(nd), key=lambda a: (lens[a], -a))
        mid = lo[axis] + lens[axis] // 2
        low_hi = list(hi); low_hi[axis] = mid
        high_lo = list(lo); high_lo[axis] = mid + 1
        sep_lo = list(lo); sep_lo[axis] = mid
        sep_hi = list(hi); sep_hi[axis] = mid + 1
        # pushed in reverse of the processing order
        stack.append((tuple(sep_lo), tuple(sep_hi), 1))
        stack.append((tuple(high_lo), tuple(hi), 0))
        stack.append((tuple(lo), tuple(low_hi), 0))
    assert pos == out.size
    if dof == 1:
        return out.astype(np.int32)
    return (out[:, None] * dof + np.arange(dof, dtype=np.int64)[None, :]).ravel().astype(np.int32)


def grid_edges(dims, stencil: str):
    """Undirected edges (i, j), i > j, of a box grid.

    stencil '5pt' (2D) / '7pt' (3D): axis neighbours; '27pt' (3D): all 26
    neighbours.  Edge order is deterministic: by offset, then by node id.
    """
    ids = grid_index(dims)
    nd = len(dims)
    if stencil in ("5pt", "7pt"):
        offsets = [tuple(1 if b == a else 0 for b in range(nd)) for a in range(nd)]
    elif stencil == "27pt":
        offsets = []
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    o = (dx, dy, dz)
                    if o > (0, 0, 0):  # one of each +/- pair
                        offsets.append(o)
    else:
        raise ValueError(stencil)
    src, dst = [], []
    for off in offsets:
        # ids array is indexed [z][y][x] (reversed dims)
        sl_a, sl_b = [], []
        for a in reversed(range(nd)):
            o = off[a]
            if o >= 0:
                sl_a.append(slice(0, dims[a] - o)); sl_b.append(slice(o, dims[a]))
            else:
                sl_a.append(slice(-o, dims[a])); sl_b.append(slice(0, dims[a] + o))
        a_ids = ids[tuple(sl_a)].ravel(); b_ids = ids[tuple(sl_b)].ravel()
        src.append(a_ids); dst.append(b_ids)
    a = np.concatenate(src); b = np.concatenate(dst)
    return np.maximum(a, b), np.minimum(a, b)


def lower_csc(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    """Assemble lower-triangular CSC (rows >= cols) from coordinate triples.

    Duplicate coordinates are summed; rows within a column come out sorted.
    """
    rows = np.asarray(rows, dtype=np.int64); cols = np.asarray(cols, dtype=np.int64)
    assert np.all(rows >= cols)
    key = cols * n + rows
    order = np.argsort(key, kind="stable")
    key = key[order]; vals = np.asarray(vals, dtype=np.float64)[order]
    uniq, start = np.unique(key, return_index=True)
    summed = np.add.reduceat(vals, start) if vals.size else vals
    c = uniq // n; r = uniq % n
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, c + 1, 1)
    colptr = np.cumsum(colptr)
    return colptr, r.astype(np.int32), summed


@dataclasses.dataclass
class System:
    """One SPD system A x = B in lower CSC form with its ordering."""
    name: str
    n: int
    colptr: np.ndarray
    rowidx: np.ndarray
    values: np.ndarray
    perm: np.ndarray
    B: np.ndarray            # float64[n, nrhs], column-major when viewed as B.T
    meta: dict

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    @property
    def nrhs(self) -> int:
        return int(self.B.shape[1])


def _rhs(key: int, n: int, nrhs: int) -> np.ndarray:
    u = uniform(key, n * nrhs)
    return np.ascontiguousarray((2.0 * u - 1.0).reshape(nrhs, n).T)


def laplacian(dims, stencil: str, workload: int, seed: int, *, unit: bool,
              shift: float, nrhs: int, sub: int = 0, name: str = "") -> System:
    """Scalar grid operator: A_ij = -c_ij per edge, A_ii = sum_j c_ij + shift.

    unit=True: every c_ij = 1.  Otherwise c_ij = 10**U[-2, 2) per undirected
    edge, drawn from the (workload, seed, EDGE, sub) stream.
    """
    n = int(np.prod(dims))
    hi, lo = grid_edges(dims, stencil)
    if unit:
        c = np.ones(hi.size)
    else:
        c = 10.0 ** (4.0 * uniform(stream_key(workload, seed, P_EDGE, sub), hi.size) - 2.0)
    diag = np.full(n, shift, dtype=np.float64)
    np.add.at(diag, hi, c); np.add.at(diag, lo, c)
    rows = np.concatenate([np.arange(n), hi]); cols = np.concatenate([np.arange(n), lo])
    vals = np.concatenate([diag, -c])
    colptr, rowidx, values = lower_csc(n, rows, cols, vals)
    return System(name or f"{stencil}-{'x'.join(map(str, dims))}", n, colptr, rowidx, values,
                  nd_perm(dims), _rhs(stream_key(workload, seed, P_RHS, sub), n, nrhs),
                  {"dims": tuple(dims), "stencil": stencil, "shift": shift, "seed": seed})


def _rotations(key: int, count: int) -> np.ndarray:
    """Uniform random rotations: sign-fixed QR of 3x3 Gaussian matrices.

    Gaussians by Box-Muller from the uniform stream.
    """
    u = uniform(key, count * 18).reshape(count, 9, 2)
    g = np.sqrt(-2.0 * np.log1p(-u[..., 0])) * np.cos(2.0 * np.pi * u[..., 1])
    q, r = np.linalg.qr(g.reshape(count, 3, 3))
    s = np.sign(np.diagonal(r, axis1=1, axis2=2))
    s[s == 0] = 1.0
    q = q * s[:, None, :]
    det = np.linalg.det(q)
    q[det < 0, :, 0] *= -1.0
    return q


def elasticity27(dims, workload: int, seed: int, *, kappa: float, nrhs: int,
                 power_iters: int = 100) -> System:
    """3-dof-per-point operator on the 27-point stencil of a box grid.

    Each edge e carries K_e = Q_e diag(10**U[-2,2) x3) Q_e^T with Q_e a
    uniform random rotation; A_ij = -K_e, A_ii = sum_e K_e + sigma I.  The
    block Laplacian is PSD with the three rigid translations as null space, so
    lambda_min(A) = sigma; sigma = lambda_max_est / kappa with lambda_max_est
    from ``power_iters`` seeded power iterations on the block Laplacian.
    """
    import scipy.sparse as sp
    npts = int(np.prod(dims)); n = 3 * npts
    hi, lo = grid_edges(dims, "27pt")
    ne = hi.size
    lam = 10.0 ** (4.0 * uniform(stream_key(workload, seed, P_EIG), ne * 3).reshape(ne, 3) - 2.0)
    Q = _rotations(stream_key(workload, seed, P_ROT), ne)
    K = np.einsum("eik,ek,ejk->eij", Q, lam, Q)
    K = 0.5 * (K + K.transpose(0, 2, 1))
    # block Laplacian as coordinate triples (full, for the power iteration)
    di = np.arange(3)
    bi, bj = np.meshgrid(di, di, indexing="ij")
    bi = bi.ravel(); bj = bj.ravel()
    Kf = K.reshape(ne, 9)
    r_off = (3 * hi[:, None] + bi[None, :]).ravel(); c_off = (3 * lo[:, None] + bj[None, :]).ravel()
    v_off = (-Kf).ravel()
    diag_blocks = np.zeros((npts, 9))
    np.add.at(diag_blocks, hi, Kf); np.add.at(diag_blocks, lo, Kf)
    r_d = (3 * np.arange(npts)[:, None] + bi[None, :]).ravel()
    c_d = (3 * np.arange(npts)[:, None] + bj[None, :]).ravel()
    v_d = diag_blocks.ravel()
    Lap = sp.coo_matrix((np.concatenate([v_d, v_off, v_off]),
                         (np.concatenate([r_d, r_off, c_off]), np.concatenate([c_d, c_off, r_off]))),
                        shape=(n, n)).tocsr()
    x = 2.0 * uniform(stream_key(workload, seed, P_POWER), n) - 1.0
    lam_max = 0.0
    for _ in range(power_iters):
        y = Lap @ x
        lam_max = float(np.linalg.norm(y) / np.linalg.norm(x))
        x = y / np.linalg.norm(y)
    sigma = lam_max / kappa
    rows_all = np.concatenate([r_d, r_off]); cols_all = np.concatenate([c_d, c_off])
    vals_all = np.concatenate([v_d + np.where(bi == bj, sigma, 0.0)[None, :].repeat(npts, 0).ravel(), v_off])
    keep = rows_all >= cols_all
    colptr, rowidx, values = lower_csc(n, rows_all[keep], cols_all[keep], vals_all[keep])
    return System(f"elast27x3-{'x'.join(map(str, dims))}", n, colptr, rowidx, values,
                  nd_perm(dims, dof=3), _rhs(stream_key(workload, seed, P_RHS), n, nrhs),
                  {"dims": tuple(dims), "stencil": "27pt", "dof": 3, "sigma": sigma,
                   "lambda_max_est": lam_max, "kappa_target": kappa, "seed": seed})


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

W_GRID2D_64, W_GRID3D_60, W_ELAST_48, W_BATCH_512, W_SERVE = 1, 2, 3, 4, 5


def grid2d_unit(k: int = 64, seed: int = 0, nrhs: int = 1) -> System:
    """2D 5-point Laplacian, off-diagonals -1, diagonal = degree + 1e-2."""
    return laplacian((k, k), "5pt", W_GRID2D_64, seed, unit=True, shift=1e-2, nrhs=nrhs)


def grid3d_cond(k: int = 60, seed: int = 0, nrhs: int = 1, shift: float = 1e-6) -> System:
    """3D 7-point operator, conductances log-uniform in [1e-2, 1e2], diag shift 1e-6."""
    return laplacian((k, k, k), "7pt", W_GRID3D_60, seed, unit=False, shift=shift, nrhs=nrhs)


def elast48(k: int = 48, seed: int = 0, nrhs: int = 4, kappa: float = 1e8) -> System:
    return elasticity27((k, k, k), W_ELAST_48, seed, kappa=kappa, nrhs=nrhs)


def batch_specs(count: int = 512, seed: int = 0):
    """(kind, side) of each system of the uneven batch.

    kind is '2d' or '3d' with probability 1/2 each; side is uniform on
    [32, 200] for 2D and [10, 34] for 3D, so n spans about 1k to 40k.
    """
    kind_u = uniform(stream_key(W_BATCH_512, seed, P_KIND), count)
    side_u = uniform(stream_key(W_BATCH_512, seed, P_SIDE), count)
    specs = []
    for i in range(count):
        if kind_u[i] < 0.5:
            specs.append(("2d", 32 + int(side_u[i] * 169)))
        else:
            specs.append(("3d", 10 + int(side_u[i] * 25)))
    return specs


def batch_system(i: int, kind: str, side: int, seed: int = 0, nrhs: int = 16,
                 workload: int = W_BATCH_512, shift: float = 1e-2) -> System:
    if kind == "2d":
        return laplacian((side, side), "5pt", workload, seed, unit=False, shift=shift, nrhs=nrhs,
                         sub=i, name=f"b{i}-5pt-{side}^2")
    return laplacian((side, side, side), "7pt", workload, seed, unit=False, shift=shift, nrhs=nrhs,
                     sub=i, name=f"b{i}-7pt-{side}^3")


def batch512(count: int = 512, seed: int = 0, nrhs: int = 16):
    return [batch_system(i, k, s, seed, nrhs) for i, (k, s) in enumerate(batch_specs(count, seed))]


def serving_requests(count: int, rate_hz: float, seed: int = 0):
    """Poisson arrivals of factor-then-solve requests.

    Each request: arrival time (exponential gaps at ``rate_hz``), and kind:
    30% re-solve of a resident factor with 8 RHS, otherwise a factor+solve of
    a new system drawn from the uneven batch mix (5% of those a 3D 7-point
    50^3 grid).
    """
    gaps = -np.log1p(-uniform(stream_key(W_SERVE, seed, P_ARRIVAL), count)) / rate_hz
    t = np.cumsum(gaps)
    mix = uniform(stream_key(W_SERVE, seed, P_MIX), count * 3).reshape(count, 3)
    reqs = []
    for i in range(count):
        if mix[i, 0] < 0.3:
            reqs.append({"id": i, "t": float(t[i]), "kind": "resolve", "pick": float(mix[i, 1]), "nrhs": 8})
        elif mix[i, 1] < 0.05:
            reqs.append({"id": i, "t": float(t[i]), "kind": "factor", "sys": ("3d", 50), "nrhs": 8})
        else:
            kind = "2d" if mix[i, 2] < 0.5 else "3d"
            u = (mix[i, 2] * 2.0) % 1.0
            side = 32 + int(u * 169) if kind == "2d" else 10 + int(u * 25)
            reqs.append({"id": i, "t": float(t[i]), "kind": "factor", "sys": (kind, side), "nrhs": 8})
    return reqs


def random_spd_pattern(n: int, density: float, seed: int, workload: int = 99):
    """Small random SPD matrix (diagonally dominant) for brute-force checks."""
    u = uniform(stream_key(workload, seed, P_EDGE), n * n).reshape(n, n)
    mask = np.tril(u < density, -1)
    r, c = np.nonzero(mask)
    vals = -(0.5 + uniform(stream_key(workload, seed, P_EIG), r.size))
    diag = np.ones(n)
    np.add.at(diag, r, -vals); np.add.at(diag, c, -vals)
    rows = np.concatenate([np.arange(n), r]); cols = np.concatenate([np.arange(n), c])
    colptr, rowidx, values = lower_csc(n, rows, cols, np.concatenate([diag, vals]))
    return colptr, rowidx, values
