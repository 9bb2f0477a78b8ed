"""Flat host description of a built H^2 representation.

Every array is plain NumPy in the layout the C-ABI's host description takes
(pointers to these arrays are handed across unchanged):

* complex values are complex128 (interleaved re, im);
* matrices are column major; blocks are concatenated at int64 element offsets;
* clusters are numbered breadth first; vectors are in tree order inside the
  representation, `perm[p]` giving the caller's voxel index at position p.

Per cluster c: level, parent, begin/end (tree positions), first_child, nchild,
rank k_c.  Leaf bases V_c (#c x k_c) sit at basis_off[c] (-1 if none);
transfer matrices T_c (k_c x k_parent) at transfer_off[c] (-1 if none);
far pairs (t, s) sorted by (level(t), t, s) with coupling S_ts (k_t x k_s) at
far_off; near pairs sorted by (t, s) with G_ts (#t x #s) at near_off.

The operator applied is Z x = x + sigma * k^2 * V * (G (x) I_ncomp)(chi . x)
with unknown index ncomp*i + c for voxel i, component c.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class H2Desc:
    n_vox: int
    ncomp: int
    perm: np.ndarray
    level: np.ndarray
    parent: np.ndarray
    begin: np.ndarray
    end: np.ndarray
    first_child: np.ndarray
    nchild: np.ndarray
    rank: np.ndarray
    basis_off: np.ndarray
    basis: np.ndarray
    transfer_off: np.ndarray
    transfer: np.ndarray
    far_t: np.ndarray
    far_s: np.ndarray
    far_off: np.ndarray
    coupling: np.ndarray
    near_t: np.ndarray
    near_s: np.ndarray
    near_off: np.ndarray
    near: np.ndarray
    chi: np.ndarray
    k: float
    volume: float
    sigma: float
    meta: dict = field(default_factory=dict)

    @property
    def n_clusters(self) -> int:
        return int(self.level.shape[0])

    @property
    def n_far(self) -> int:
        return int(self.far_t.shape[0])

    @property
    def n_near(self) -> int:
        return int(self.near_t.shape[0])

    @property
    def N(self) -> int:
        return self.n_vox * self.ncomp

    def size(self, c):
        return self.end[c] - self.begin[c]

    def basis_of(self, c: int) -> np.ndarray:
        n = int(self.end[c] - self.begin[c])
        k = int(self.rank[c])
        o = int(self.basis_off[c])
        return self.basis[o:o + n * k].reshape(k, n).T

    def transfer_of(self, c: int) -> np.ndarray:
        p = int(self.parent[c])
        kc, kp = int(self.rank[c]), int(self.rank[p])
        o = int(self.transfer_off[c])
        return self.transfer[o:o + kc * kp].reshape(kp, kc).T

    def coupling_of(self, i: int) -> np.ndarray:
        t, s = int(self.far_t[i]), int(self.far_s[i])
        kt, ks = int(self.rank[t]), int(self.rank[s])
        o = int(self.far_off[i])
        return self.coupling[o:o + kt * ks].reshape(ks, kt).T

    def near_of(self, i: int) -> np.ndarray:
        t, s = int(self.near_t[i]), int(self.near_s[i])
        nt, ns = int(self.end[t] - self.begin[t]), int(self.end[s] - self.begin[s])
        o = int(self.near_off[i])
        return self.near[o:o + nt * ns].reshape(ns, nt).T

    def nbytes_algorithmic(self, bytes_per_complex: int = 16, ncols: int | None = None) -> int:
        """Bytes the matvec must move: every stored block once, plus x read and y written."""
        if ncols is None:
            ncols = self.ncomp
        blocks = self.near.size + self.coupling.size + self.basis.size + self.transfer.size
        vec = 2 * self.n_vox * ncols
        return int((blocks + vec) * bytes_per_complex)

    def flops_algorithmic(self, ncols: int | None = None) -> int:
        """Real flops of one product with `ncols` columns (8 per complex multiply-add)."""
        if ncols is None:
            ncols = self.ncomp
        return int(8 * ncols * (self.near.size + self.coupling.size
                                + 2 * self.basis.size + 2 * self.transfer.size))

    def save_dir(self, path: str) -> None:
        """One .npy per array (loadable memory-mapped), plus scalars and meta as JSON."""
        import json
        import os
        os.makedirs(path, exist_ok=True)
        scal = {}
        for k in self.__dataclass_fields__:
            v = getattr(self, k)
            if k == "meta":
                continue
            if isinstance(v, np.ndarray):
                np.save(os.path.join(path, k + ".npy"), v)
            else:
                scal[k] = v
        with open(os.path.join(path, "desc.json"), "w") as f:
            json.dump({"scalars": scal, "meta": self.meta}, f)

    @staticmethod
    def load_dir(path: str, mmap: bool = True) -> "H2Desc":
        import json
        import os
        with open(os.path.join(path, "desc.json")) as f:
            j = json.load(f)
        kw = dict(j["scalars"])
        for k in H2Desc.__dataclass_fields__:
            if k == "meta" or k in kw:
                continue
            kw[k] = np.load(os.path.join(path, k + ".npy"), mmap_mode="r" if mmap else None)
        kw["meta"] = j["meta"]
        return H2Desc(**kw)

    def save(self, path: str) -> None:
        arrs = {k: getattr(self, k) for k in self.__dataclass_fields__ if k != "meta"}
        arrs = {k: (np.asarray(v)) for k, v in arrs.items()}
        np.savez(path, **arrs, meta_json=np.array(__import__("json").dumps(self.meta)))

    @staticmethod
    def load(path: str) -> "H2Desc":
        import json
        z = np.load(path, allow_pickle=False)
        kw = {}
        for k in H2Desc.__dataclass_fields__:
            if k == "meta":
                continue
            v = z[k]
            if k in ("n_vox", "ncomp"):
                v = int(v)
            elif k in ("k", "volume", "sigma"):
                v = float(v)
            kw[k] = v
        kw["meta"] = json.loads(str(z["meta_json"]))
        return H2Desc(**kw)
