"""O(N) storage and product work of the representation (the paper's complexity claim,
Sec. IV.B and Sec. V): on rods of growing length at a fixed voxel size the bytes and flops
per unknown settle to a constant and the ranks stay bounded."""
import numpy as np

from h2gen.construct import build_h2
from h2gen.geometry import box


def test_storage_and_work_per_unknown_settle():
    per_b, per_f, ranks = [], [], []
    for L in (64, 128, 256, 512, 1024):
        g = box((L, 4, 4), 1.0 / 16, eps=(2.0, 6.0), seed=7)
        d = build_h2(g, eps=1e-4)
        N = 3 * g.n_vox
        per_b.append(d.nbytes_algorithmic() / N)
        per_f.append(d.flops_algorithmic() / N)
        ranks.append(int(np.max(d.rank)))
    per_b, per_f = np.array(per_b), np.array(per_f)
    # 16x more unknowns, less than 15% more per unknown; the growth steps shrink
    assert per_b[-1] < 1.15 * per_b[0] and per_f[-1] < 1.2 * per_f[0]
    steps = np.diff(per_b)
    assert np.all(steps[1:] < steps[:-1])
    assert max(ranks) - min(ranks) <= 2
