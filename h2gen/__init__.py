"""Seeded input generators for the H^2 VIE hot path.

This package produces every input that both the HIP path and the CPU oracle
consume: voxel geometries and permittivities, right-hand sides, the cluster
tree, the strong-admissibility block partition (Sec. III.A, eq. (4)) and the
minimal-rank H^2 representation built by the paper's two-stage construction
(Sec. III.B-C, eqs. (5)-(18)).  The construction is an input generator here:
the hot path (the matvec of Sec. IV.B and the Krylov solver around it) is not
implemented in this package, and nothing in it is shared with either side's
arithmetic.  Both consume the flat arrays of :class:`h2gen.desc.H2Desc`.
"""

from .geometry import Geometry, cube, slab, uneven_cubes, paper_rod, paper_slab, paper_cube_array  # noqa: F401
from .tree import ClusterTree, build_tree  # noqa: F401
from .partition import Partition, build_partition  # noqa: F401
from .desc import H2Desc  # noqa: F401
from .construct import build_h2  # noqa: F401
from .rhs import random_vector, plane_wave, plane_wave_dir, paper_excitation  # noqa: F401
