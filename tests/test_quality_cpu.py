"""Host-side checks of the quality harness's measures: PSNR against its closed
form, and tie-aware recall@K against brute-force nearest neighbours on tiny
clouds."""
import itertools

import numpy as np
import pytest

pytest.importorskip("scipy")

from paper_2401_09721_amd import quality  # noqa: E402


def test_psnr_closed_form():
    ref = np.zeros((4, 3))
    x = np.full((4, 3), 5.0)  # MSE 25
    assert quality.psnr(x, ref) == pytest.approx(10 * np.log10(255.0 ** 2 / 25.0))
    x[0, 0] = 15.0  # MSE (11*25 + 225) / 12
    assert quality.psnr(x, ref) == pytest.approx(10 * np.log10(255.0 ** 2 * 12 / (11 * 25 + 225)))
    assert quality.psnr(ref, ref) == float("inf")


def brute_knn(xyz, k):
    d2 = ((xyz[:, None, :].astype(np.int64) - xyz[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.iinfo(np.int64).max)
    order = np.argsort(d2, axis=1, kind="stable")[:, :k]
    return order.astype(np.int32), np.sort(d2, axis=1)[:, k - 1]


@pytest.mark.parametrize("seed", [0, 1])
def test_recall_of_exact_knn_is_one_and_drops_per_wrong_slot(seed):
    rng = np.random.default_rng(seed)
    xyz = np.unique(rng.integers(0, 12, size=(300, 3)), axis=0).astype(np.int32)
    n, k = xyz.shape[0], 6
    col, kth = brute_knn(xyz, k)
    rows = np.arange(n)
    assert np.array_equal(quality.exact_kth_dist2(xyz, rows, k), kth)
    assert quality.knn_recall(xyz, col, rows, k) == 1.0
    # replace one neighbour of point 0 by its farthest point, and empty one slot of point 1
    bad = col.copy()
    d0 = ((xyz.astype(np.int64) - xyz[0]) ** 2).sum(-1)
    bad[0, 2] = int(np.argmax(d0))
    bad[1, 5] = -1
    assert quality.knn_recall(xyz, bad, rows, k) == pytest.approx(1.0 - 2.0 / (k * n))
    # the point itself is never a hit
    bad[2, 0] = 2
    assert quality.knn_recall(xyz, bad, rows, k) == pytest.approx(1.0 - 3.0 / (k * n))


def test_recall_counts_any_of_equally_near_sets():
    # the centre of a 3x3x3 block has six neighbours at squared distance 1;
    # with K = 4 any four of them are an exact answer
    xyz = np.array(list(itertools.product(range(3), repeat=3)), np.int32)
    centre = 13
    assert tuple(xyz[centre]) == (1, 1, 1)
    unit = [i for i in range(27) if ((xyz[i] - xyz[centre]) ** 2).sum() == 1]
    assert len(unit) == 6
    col = np.full((27, 4), -1, np.int32)
    for pick in (unit[:4], unit[2:]):
        col[centre] = pick
        assert quality.knn_recall(xyz, col, [centre], 4) == 1.0
    corner = [i for i in range(27) if ((xyz[i] - xyz[centre]) ** 2).sum() == 3][0]
    col[centre] = unit[:3] + [corner]
    assert quality.knn_recall(xyz, col, [centre], 4) == 0.75


def test_oracle_more_directions_never_give_a_farther_row():
    # the L = 8 scan directions start with the L = 4 ones, so the candidate set
    # only grows and the K kept neighbours are at least as near, slot by slot
    import oracle as O
    from paper_2401_09721_amd import synth

    c = synth.random_shapes_cloud(seed=3, target=3000)
    d = []
    for L in (4, 8):
        col, dist2 = O.slg_graph(c.xyz, 8, L, 4, 8)[:2]
        d.append(np.sort(np.where(np.asarray(col) >= 0, dist2, np.iinfo(np.int64).max), axis=1))
    assert (d[1] <= d[0]).all()
    assert (d[1] < d[0]).any()
