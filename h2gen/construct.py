"""Minimal-rank H^2 construction (Sec. III.B-C), used as the input generator.

Stage I (eqs. (5)-(7)): for every cluster t with admissible blocks at its
level, ACA + reduced SVD of the grouped block row G^t gives A_t B_t^T and the
k x k Gram K_t = B_t^T conj(B_t).

Stage II:
* leaf bases (eqs. (10)-(12)): G2 = A_t K_t A_t^H + sum over ancestors j of
  A_j|_t K_j A_j|_t^H; its leading eigenvectors (eigenvalues d_i > eps^2 d_1,
  i.e. singular values above eps * sigma_1) form V_t;
* transfer matrices (eqs. (13)-(16)), bottom up: every factor F covering t is
  projected onto the children's bases, F_small = [V_c1^H F|_c1; ...]; the
  k x k Gram sum F_small K F_small^H is eigendecomposed and truncated, and the
  row blocks of the kept eigenvectors are the transfers T_ci;
* couplings (eqs. (17)-(18)): S_ts = (V_t^H A_t) (V_s^H B_t|_s)^T.

Projections onto nested bases use the recursion V_p^H F|_p =
sum_c T_c^H (V_c^H F|_c).  Near (inadmissible) blocks are the dense kernel
entries.  Complex bases stay complex (V^H V = I).
"""

from __future__ import annotations

import mmap
import multiprocessing as mp
import os
import sys
import time

import numpy as np

from .aca import aca_partial, rsvd_truncate
from .desc import H2Desc
from .geometry import Geometry
from .partition import build_partition
from .tree import build_tree


def _workers(n=None):
    if n:
        return n
    env = os.environ.get("H2GEN_WORKERS")
    if env:
        return int(env)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


# Work functions run in forked worker processes; they read the state of the
# current build from this module-level slot, inherited at fork time, and may
# keep per-item results in _LOCAL (worker memory) for a later phase.
_STATE = {}
_LOCAL = {}


def _worker_loop(conn):
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        while True:
            msg = conn.recv()
            if msg is None:
                break
            name, item, payload = msg
            if payload is not None:
                _STATE.update(payload)
            try:
                conn.send((True, _STATE[name](item) if name else None))
            except Exception as e:  # report and keep serving
                import traceback
                conn.send((False, traceback.format_exc() + repr(e)))
    conn.close()


class _Pool:
    """Forked workers pulling items one at a time; each worker keeps its own
    _LOCAL between phases, and `owner[item]` records which worker ran it."""

    def __init__(self, nproc: int):
        self.nproc = nproc
        self.conns, self.procs = [], []
        if nproc <= 1:
            return
        ctx = mp.get_context("fork")
        for _ in range(nproc):
            a, b = ctx.Pipe()
            p = ctx.Process(target=_worker_loop, args=(b,), daemon=True)
            p.start()
            b.close()
            self.conns.append(a)
            self.procs.append(p)

    def map(self, name, items, payload=None, owner=None, assign=None):
        """Results in item order.  assign[item] pins an item to a worker."""
        items = list(items)
        if self.nproc <= 1:
            if payload:
                _STATE.update(payload)
            from threadpoolctl import threadpool_limits
            with threadpool_limits(1):
                return [_STATE[name](x) for x in items]
        from multiprocessing.connection import wait
        res = [None] * len(items)
        queues = [[] for _ in range(self.nproc)]
        shared = []
        for idx, x in enumerate(items):
            if assign is not None:
                queues[assign[x]].append(idx)
            else:
                shared.append(idx)
        busy = {}
        fresh = set(range(self.nproc))

        def feed(w):
            q = queues[w] if queues[w] else shared
            if not q:
                return False
            idx = q.pop(0)
            pl = payload if w in fresh else None
            fresh.discard(w)
            self.conns[w].send((name, items[idx], pl))
            busy[w] = idx
            return True

        for w in range(self.nproc):
            if not feed(w) and payload is not None:
                self.conns[w].send((None, None, payload))
                fresh.discard(w)
                busy[w] = -1
        while busy:
            ready = wait([self.conns[w] for w in busy])
            for cn in ready:
                w = self.conns.index(cn)
                ok, val = cn.recv()
                idx = busy.pop(w)
                if not ok:
                    raise RuntimeError(val)
                if idx >= 0:
                    res[idx] = val
                    if owner is not None:
                        owner[items[idx]] = w
                feed(w)
        return res

    def close(self):
        for c in self.conns:
            try:
                c.send(None)
            except (BrokenPipeError, OSError):
                pass
        for p in self.procs:
            p.join(timeout=10)
        self.conns, self.procs = [], []


def _pmap(name, items, nproc):
    """Map _STATE[name] over items in freshly forked processes (results in order)."""
    items = list(items)
    pool = _Pool(nproc if len(items) > 1 else 1)
    try:
        return pool.map(name, items)
    finally:
        pool.close()


def _shared_array(n: int, dtype=np.complex128) -> np.ndarray:
    """Anonymous MAP_SHARED array: writes from forked workers land in the parent."""
    nbytes = max(1, int(n) * np.dtype(dtype).itemsize)
    buf = mmap.mmap(-1, nbytes, flags=mmap.MAP_SHARED | mmap.MAP_ANONYMOUS)
    return np.frombuffer(buf, dtype=dtype, count=int(n))


class _Kernel:
    """Entries of G between tree positions through the distance table."""

    def __init__(self, geom: Geometry, coords: np.ndarray):
        self.tab = geom.green_table()
        self.c = coords.astype(np.int32)

    def block(self, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
        cr = self.c[rows]
        cc = self.c[cols]
        d = cr[:, None, 0] - cc[None, :, 0]
        d2 = d * d
        d = cr[:, None, 1] - cc[None, :, 1]
        d2 += d * d
        d = cr[:, None, 2] - cc[None, :, 2]
        d2 += d * d
        return self.tab[d2]

    def row(self, p: int, cols_c: np.ndarray) -> np.ndarray:
        d = cols_c - self.c[p]
        d *= d
        return self.tab[d.sum(1)]


def _ranges(begin, end, items):
    return np.concatenate([np.arange(begin[s], end[s]) for s in items]) if len(items) else np.zeros(0, np.int64)


def _truncate_eigh(G2: np.ndarray, eps: float):
    w, P = np.linalg.eigh(G2)
    w = w[::-1]
    P = P[:, ::-1]
    if w.size == 0 or w[0] <= 0.0:
        return P[:, :0]
    k = int(np.count_nonzero(w > (eps * eps) * w[0]))
    return np.ascontiguousarray(P[:, :k])


def _stage1(st, t):
    """ACA + r-SVD of the grouped block row of cluster t: (A, B, K)."""
    tree, ker, partners = st["tree"], st["ker"], st["partners"]
    rows = np.arange(tree.begin[t], tree.end[t])
    cols = _ranges(tree.begin, tree.end, partners[t])
    cols_c = ker.c[cols]
    U, V = aca_partial(lambda i: ker.row(int(rows[i]), cols_c),
                       lambda j: ker.block(rows, cols[j:j + 1])[:, 0], rows.size, cols.size, st["eps_aca"])
    return rsvd_truncate(U, V, st["eps"])


def _project(st, cl, F):
    """V_cl^H F for F with #cl rows, through the nested basis of cl."""
    tree, rank = st["tree"], st["rank"]
    if tree.nchild[cl] == 0:
        return st["Vb"][cl].conj().T @ F
    acc = np.zeros((int(rank[cl]), F.shape[1]), np.complex128)
    for c in tree.children(cl):
        if rank[c] == 0:
            continue
        o = int(tree.begin[c] - tree.begin[cl])
        acc += st["T"][c].conj().T @ _project(st, c, F[o:o + int(tree.end[c] - tree.begin[c])])
    return acc


def _ph_stage1(t):
    st = _STATE["st"]
    A, B, K = _stage1(st, t)
    if st["keep_b"]:
        _LOCAL[t] = B
    return A, K


def _ph_couplings(t):
    """Couplings of row cluster t: list of S_ts (k_t x k_s) in partner order."""
    st = _STATE["st"]
    B = _LOCAL.pop(t, None)
    if B is None:
        B = _stage1(st, t)[1]          # same arithmetic as Stage I
    PA = st["PA"][t]
    size = st["tree"].end - st["tree"].begin
    out = []
    o = 0
    for s in st["partners"][t]:
        ns = int(size[s])
        out.append(PA @ _project(st, int(s), B[o:o + ns]).T)
        o += ns
    return out


def _mem_available() -> float:
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemAvailable:"):
                    return float(line.split()[1]) * 1024.0
    except OSError:
        pass
    return 8e9


def build_h2(geom: Geometry, leaf_size: int = 64, eta: float = 1.0, eps: float = 1e-3,
             eps_aca: float | None = None, workers: int | None = None,
             verbose: bool = False, with_near: bool = True, keep_b_bytes: float | None = None) -> H2Desc:
    """Build the H^2 representation of G for `geom` (see the module docstring)."""
    t0 = time.time()
    nproc = _workers(workers)
    if eps_aca is None:
        eps_aca = eps / 10.0
    tree = build_tree(geom.shape, leaf_size)
    part = build_partition(tree, eta)
    ker = _Kernel(geom, tree.coords)
    ncl = tree.n_clusters
    leaf = tree.nchild == 0
    size = tree.end - tree.begin

    # partners R_t in far-list order (the far list is sorted by (level(t), t, s))
    order = np.argsort(part.far_t, kind="stable")
    cuts = np.searchsorted(part.far_t[order], np.arange(ncl + 1))
    fs = part.far_s[order]
    partners = [fs[cuts[c]:cuts[c + 1]] for c in range(ncl)]
    first = cuts[:-1].astype(np.int64)           # far index of (t, first partner)
    has_blocks = np.array([len(p) > 0 for p in partners])
    work = [c for c in range(ncl) if has_blocks[c]]
    ncols = {c: int(size[partners[c]].sum()) for c in work}
    work.sort(key=lambda c: -int(size[c]) * ncols[c])
    # B_t is (#cols x k) per cluster; keep it in the workers when it fits
    est_b = sum(ncols[c] * 24 * 16 for c in work)   # B_t is #cols x k_t, k_t ~ 10-36 here
    if keep_b_bytes is None:
        keep_b_bytes = min(0.35 * _mem_available(), 120e9)
    keep_b = est_b <= keep_b_bytes
    if verbose:
        print(f"[h2gen] {geom.name}: {ncl} clusters, {part.n_far} far, {part.n_near} near, "
              f"{nproc} workers, keep B: {keep_b} (~{est_b/1e9:.1f} GB of {keep_b_bytes/1e9:.0f} GB budget)  "
              f"{time.time()-t0:.1f}s", file=sys.stderr, flush=True)

    st = dict(tree=tree, ker=ker, partners=partners, eps=eps, eps_aca=eps_aca, keep_b=keep_b)
    _STATE.clear()
    _LOCAL.clear()
    _STATE.update(st=st, stage1=_ph_stage1, couplings=_ph_couplings)
    pool = _Pool(nproc)
    try:
        # ---- Stage I: A_t, K_t in the parent; B_t stays with the worker that made it
        owner = {}
        A = [None] * ncl
        K = [None] * ncl
        for c, (a, kk) in zip(work, pool.map("stage1", work, owner=owner)):
            A[c] = a
            K[c] = kk
        if verbose:
            print(f"[h2gen] stage I {time.time()-t0:.1f}s", file=sys.stderr, flush=True)

        # ---- Stage II: terms covering each cluster (itself and ancestors with blocks)
        terms = [None] * ncl
        for c in range(ncl):
            p = int(tree.parent[c])
            base = terms[p] if p >= 0 else []
            terms[c] = (base + [c]) if has_blocks[c] else list(base)
        rank = np.zeros(ncl, np.int64)
        Vb = [None] * ncl       # leaf bases V_t
        T = [None] * ncl        # transfer T_c (k_c x k_parent)
        proj = [None] * ncl     # dict j -> V_c^H A_j|_c

        def leaf_basis(c):
            tm = terms[c]
            n = int(size[c])
            if not tm:
                return np.zeros((n, 0), np.complex128), {}
            G2 = np.zeros((n, n), np.complex128)
            rows = {}
            for j in tm:
                o = int(tree.begin[c] - tree.begin[j])
                Aj = A[j][o:o + n]
                rows[j] = Aj
                G2 += (Aj @ K[j]) @ Aj.conj().T
            V = _truncate_eigh(G2, eps)
            return V, {j: V.conj().T @ rows[j] for j in tm}

        def inner(p):
            tm = terms[p]
            if not tm:
                return None, {}
            kids = list(tree.children(p))
            Fs = {j: np.concatenate([proj[c][j] for c in kids], axis=0) for j in tm}
            ksum = next(iter(Fs.values())).shape[0]
            G2 = np.zeros((ksum, ksum), np.complex128)
            for j in tm:
                G2 += (Fs[j] @ K[j]) @ Fs[j].conj().T
            P = _truncate_eigh(G2, eps)
            return P, {j: P.conj().T @ Fs[j] for j in tm}

        _STATE.update(leaf_basis=leaf_basis, inner=inner)
        leaves = np.nonzero(leaf)[0]
        for c, (V, pr) in zip(leaves, _pmap("leaf_basis", leaves, nproc)):
            Vb[c] = V
            rank[c] = V.shape[1]
            proj[c] = pr
        for lev in range(tree.depth - 1, -1, -1):
            nodes = [int(c) for c in np.nonzero((tree.level == lev) & ~leaf)[0]]
            for p, (P, pr) in zip(nodes, _pmap("inner", nodes, nproc if len(nodes) > 64 else 1)):
                kids = list(tree.children(p))
                if P is None:
                    rank[p] = 0
                    proj[p] = {}
                else:
                    rank[p] = P.shape[1]
                    o = 0
                    for c in kids:
                        kc = int(rank[c])
                        T[c] = np.ascontiguousarray(P[o:o + kc])
                        o += kc
                    proj[p] = pr
                for c in kids:   # children keep only their own projection V_c^H A_c
                    proj[c] = {c: proj[c][c]} if c in proj[c] else {}
        if verbose:
            print(f"[h2gen] stage II bases {time.time()-t0:.1f}s; ranks " +
                  ", ".join(f"L{l}:{rank[tree.level == l].min()}-{rank[tree.level == l].max()}"
                            for l in range(tree.depth + 1)), file=sys.stderr, flush=True)

        # ---- couplings S_ts = (V_t^H A_t)(V_s^H B_t|_s)^T on the workers holding B_t
        far_t, far_s = part.far_t, part.far_s
        far_sizes = rank[far_t] * rank[far_s]
        far_off = np.concatenate([[0], np.cumsum(far_sizes)[:-1]]).astype(np.int64)
        coupling = np.zeros(int(far_sizes.sum()), np.complex128)
        PA = {c: proj[c][c] for c in work}
        payload = dict(st=dict(st, rank=rank, Vb=Vb, T=T, PA=PA))
        assign = owner if keep_b else None
        for t, blocks in zip(work, pool.map("couplings", work, payload=payload, assign=assign)):
            i = int(first[t])
            for S in blocks:
                o = int(far_off[i])
                coupling[o:o + S.size] = S.reshape(-1, order="F")
                i += 1
        if verbose:
            print(f"[h2gen] couplings {time.time()-t0:.1f}s ({coupling.nbytes/1e9:.2f} GB)", file=sys.stderr, flush=True)
    finally:
        pool.close()

    # ---- flat bases and transfers
    basis_off = np.full(ncl, -1, np.int64)
    chunks, o = [], 0
    for c in leaves:
        if rank[c] > 0:
            basis_off[c] = o
            chunks.append(Vb[c].reshape(-1, order="F"))
            o += Vb[c].size
    basis = np.concatenate(chunks) if chunks else np.zeros(0, np.complex128)
    transfer_off = np.full(ncl, -1, np.int64)
    chunks, o = [], 0
    for c in range(ncl):
        if T[c] is not None and T[c].size:
            transfer_off[c] = o
            chunks.append(T[c].reshape(-1, order="F"))
            o += T[c].size
    transfer = np.concatenate(chunks) if chunks else np.zeros(0, np.complex128)

    # ---- near blocks (dense kernel entries), written in place by forked workers
    near_t, near_s = part.near_t, part.near_s
    nsz = size[near_t] * size[near_s]
    near_off = np.concatenate([[0], np.cumsum(nsz)[:-1]]).astype(np.int64)
    if with_near:
        near = _shared_array(int(nsz.sum()))
        step = max(1, part.n_near // (nproc * 8))

        def fill(lo):
            for i in range(lo, min(lo + step, part.n_near)):
                t, s = int(near_t[i]), int(near_s[i])
                blk = ker.block(np.arange(tree.begin[t], tree.end[t]), np.arange(tree.begin[s], tree.end[s]))
                near[near_off[i]:near_off[i] + blk.size] = blk.reshape(-1, order="F")
            return None
        _STATE["near"] = fill
        _pmap("near", range(0, part.n_near, step), nproc)
    else:
        near = np.zeros(0, np.complex128)
    _STATE.clear()
    if verbose:
        print(f"[h2gen] near {time.time()-t0:.1f}s ({near.nbytes/1e9:.2f} GB)", file=sys.stderr, flush=True)

    meta = dict(name=geom.name, shape=list(geom.shape), h=geom.h, leaf_size=leaf_size, eta=eta, eps=eps,
                eps_aca=eps_aca, build_seconds=time.time() - t0, geom_meta=geom.meta)
    return H2Desc(n_vox=tree.n_vox, ncomp=3, perm=tree.perm.copy(), level=tree.level.copy(),
                  parent=tree.parent.copy(), begin=tree.begin.copy(), end=tree.end.copy(),
                  first_child=tree.first_child.copy(), nchild=tree.nchild.copy(),
                  rank=rank.astype(np.int32), basis_off=basis_off, basis=basis,
                  transfer_off=transfer_off, transfer=transfer,
                  far_t=far_t.copy(), far_s=far_s.copy(), far_off=far_off, coupling=coupling,
                  near_t=near_t.copy(), near_s=near_s.copy(), near_off=near_off, near=near,
                  chi=geom.chi.copy(), k=float(geom.k), volume=float(geom.volume), sigma=float(geom.sigma),
                  meta=meta)


def symmetrize_couplings(d: H2Desc, chunk: int = 1 << 16) -> H2Desc:
    """Return d with S_ts := (S_ts + S_st^T) / 2 and S_st := S_ts^T for every
    unordered admissible pair {t, s}.

    G is complex symmetric (its entries depend on |r - r'| only) and the product
    uses one basis per cluster for rows and columns (G^{t,s} ~ V_t S_ts V_s^T,
    eq. (8)), so S_st and S_ts^T approximate the same block; eq. (18) computes them
    from two different Stage I factorisations, and they agree to the truncation
    accuracy only.  The average keeps that accuracy and makes the stored pair exact
    transposes bit for bit, so a product may stream each unordered pair once.  The
    partition lists both orders of every admissible pair (eq. (4) is symmetric in
    t and s).  Everything else is shared with d; the coupling array is a new copy.
    """
    import dataclasses
    ncl = int(d.level.shape[0])
    far_t = d.far_t.astype(np.int64)
    far_s = d.far_s.astype(np.int64)
    key = far_t * ncl + far_s
    order = np.argsort(key, kind="stable")
    pos = np.searchsorted(key[order], far_s * ncl + far_t)
    if np.any(pos >= key.size):
        raise ValueError("far list is not symmetric")
    rev = order[pos]
    if not np.array_equal(key[rev], far_s * ncl + far_t):
        raise ValueError("far list is not symmetric")
    C = d.coupling.copy()
    rank = d.rank.astype(np.int64)
    kt, ks = rank[far_t], rank[far_s]
    first = np.nonzero(far_t < far_s)[0]
    pairs = np.stack([kt[first], ks[first]], 1)
    for a, b in np.unique(pairs, axis=0):
        idx = first[(pairs[:, 0] == a) & (pairs[:, 1] == b)]
        n_el = int(a * b)
        if n_el == 0:
            continue
        ar = np.arange(n_el, dtype=np.int64)
        for lo in range(0, idx.size, chunk):
            i = idx[lo:lo + chunk]
            j = rev[i]
            oi = d.far_off[i][:, None] + ar
            oj = d.far_off[j][:, None] + ar
            S_ts = C[oi].reshape(-1, b, a)            # [n, col, row] of the k_t x k_s block (column major)
            S_st = C[oj].reshape(-1, a, b)            # [n, col, row] of the k_s x k_t block
            M = (S_ts + S_st.transpose(0, 2, 1)) * 0.5
            C[oi] = M.reshape(-1, n_el)
            C[oj] = M.transpose(0, 2, 1).reshape(-1, n_el)
    meta = dict(d.meta)
    meta["symmetric_couplings"] = True
    return dataclasses.replace(d, coupling=C, meta=meta)
