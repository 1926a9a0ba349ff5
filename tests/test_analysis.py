"""The product's droplet statistics (paper_1803_01756_amd.analysis, scipy
labelling with the periodic x seam joined) against the oracle scripts'
plain flood fills, which write the stored droplet records the GPU runs are
compared with: the same sets, counts and centroids on random fields that
wrap across the x seam and touch both plates, and on hand-made cases."""
import numpy as np
import pytest

from oracle.crop_droplet_stats import droplet_stats
from oracle.gravity_drop import liquid_sets as oracle_sets
from paper_1803_01756_amd import analysis


def _field(seed, ny=24, nx=40, frac=0.45):
    rng = np.random.default_rng(seed)
    rho = np.where(rng.random((ny, nx)) < frac, 6.0, 0.4)
    rho[0] = rho[-1] = 0.0  # plate rows
    return rho


@pytest.mark.parametrize("seed", range(8))
def test_liquid_sets_match_oracle(seed):
    rho = _field(seed)
    a = analysis.liquid_sets(rho, 3.0)
    b = oracle_sets(rho, 3.0)
    key = lambda r: (-r[0], round(r[1], 9), round(r[2], 9))
    a, b = sorted(a, key=key), sorted(b, key=key)
    assert len(a) == len(b) > 3
    for x, y in zip(a, b):
        assert x[0] == y[0] and x[3:] == y[3:]
        assert abs(x[1] - y[1]) < 1e-12 and abs(x[2] - y[2]) < 1e-9


@pytest.mark.parametrize("seed", range(6))
def test_plate_droplets_match_oracle(seed):
    rho = _field(100 + seed, frac=0.3)
    a = analysis.droplets(rho, 3.0)
    b = droplet_stats(rho, 3.0)
    for side in ("bottom", "top"):
        assert a[side]["count"] == b[side]["count"]
        assert abs(a[side]["mean_spacing"] - b[side]["mean_spacing"]) < 1e-9
    assert a["condensed_nodes"] == b["condensed_nodes"]


def test_set_across_the_seam_is_one_set():
    rho = np.full((8, 20), 0.4)
    rho[0] = rho[-1] = 0.0
    rho[3:5, :3] = 6.0
    rho[3:5, -2:] = 6.0
    sets = analysis.liquid_sets(rho, 3.0)
    assert len(sets) == 1 and sets[0][0] == 10
    # circular mean of columns 18, 19, 0, 1, 2 is column 0
    assert abs(sets[0][2] % 20) < 1e-9 or abs(sets[0][2] - 20) < 1e-9
    assert sets[0][3:] == [0, 0]


def test_contact_flags():
    rho = np.full((10, 12), 0.4)
    rho[0] = rho[-1] = 0.0
    rho[1:4, 2] = 6.0    # on the bottom plate
    rho[6:9, 8] = 6.0    # under the top plate
    sets = sorted(analysis.liquid_sets(rho, 3.0), key=lambda r: r[1])
    assert [s[3:] for s in sets] == [[0, 1], [1, 0]]


def test_open_sets_are_not_joined_across_the_ends():
    rho = np.full((8, 20), 0.4)
    rho[0] = rho[-1] = 0.0
    rho[3:5, :3] = 6.0    # at the inlet
    rho[5:7, -2:] = 6.0   # at the outlet, on the top plate (row 6 = ny - 2)
    sets = analysis.liquid_sets_open(rho, 3.0)
    assert [s[0] for s in sets] == [6, 4]
    assert sets[0][1:] == [3.5, 1.0, 0, 0]
    assert sets[1][1:] == [5.5, 18.5, 1, 0]
