"""Host-side logic of the package that needs no GPU, checked against the oracle's own versions."""
import numpy as np
import pytest

from conftest import built
from oracle import mlp as omlp


@pytest.mark.parametrize("name", ["cube12", "box9", "cube13", "rod", "slab"])
def test_leaf_neighbors_match_oracle_halo_table(name):
    from paper_1703_01175_amd.api import leaf_neighbors
    g, d = built(name)
    tab = leaf_neighbors(d, g.shape)
    assert tab.dtype == np.int32
    assert np.array_equal(tab, omlp.halo_table(d, g.shape))
