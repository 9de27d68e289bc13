"""Input generators: reference values of the RNGs, well-formed CSR, determinism."""
import hashlib
import os
import subprocess
import sys

import numpy as np
import pytest

import graphgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_splitmix64_reference_stream():
    # SplitMix64 from state 0: the first outputs of the published reference code
    assert [graphgen.splitmix64_at(0, i) for i in range(3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_bounded_in_range_and_uniform():
    x = graphgen.bounded_outputs(7, 0, 10, 200_000)
    assert x.min() == 0 and x.max() == 9
    counts = np.bincount(x.astype(np.int64), minlength=10)
    chi2 = (((counts - 20_000) ** 2) / 20_000).sum()
    assert chi2 < 40  # 9 dof, p ~ 1e-5


def test_permutation_is_uniform_permutation():
    p = graphgen.permutation(1000, 3)
    assert sorted(p.tolist()) == list(range(1000))
    counts = {}
    for s in range(12_000):
        key = tuple(graphgen.permutation(4, s).tolist())
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 24
    exp = 12_000 / 24
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < 60  # 23 dof


def check_csr(g):
    off, col, n = g.off, g.col, g.n
    assert off[0] == 0 and (np.diff(off) >= 0).all() and off[-1] == len(col)
    rows = np.repeat(np.arange(n), np.diff(off))
    if g.vtx_ptr is not None:
        gid = np.searchsorted(g.vtx_ptr, rows, side="right") - 1
        base = g.vtx_ptr[gid]
        loc_rows = rows - base
        sizes = np.diff(g.vtx_ptr)
        assert (col >= 0).all() and (col < sizes[gid]).all()
        glob_col = col.astype(np.int64) + base
    else:
        loc_rows = rows
        assert (col >= 0).all() and (col < n).all()
        glob_col = col.astype(np.int64)
    assert (glob_col != rows).all(), "self-loop"
    key = rows.astype(np.int64) * (n + 1) + glob_col
    assert (np.diff(key) > 0).all(), "rows must be strictly ascending"
    rkey = glob_col * (n + 1) + rows
    assert np.array_equal(np.sort(rkey), key), "not symmetric"
    del loc_rows


@pytest.mark.parametrize("maker", [
    lambda: graphgen.erdos_renyi(2000, 10.0, 1),
    lambda: graphgen.chung_lu(5000, 2.1, 20.0, 2),
    lambda: graphgen.rmat(12, 16, 0.57, 0.19, 0.19, 3),
    lambda: graphgen.sbm_batch(*graphgen.sbm_shapes(20, 4, nmax=400), 0.3, 0.01, 4),
    lambda: graphgen.from_edges(6, [(0, 1), (1, 0), (2, 2), (3, 4), (4, 3), (5, 0)]),
])
def test_graphs_well_formed(maker):
    check_csr(maker())


def test_er_mean_degree():
    g = graphgen.erdos_renyi(20_000, 10.0, seed=1)
    assert abs(g.nnz / g.n - 10.0) < 0.2


def test_chung_lu_weights():
    w = graphgen.chung_lu_weights(100_000, 2.1, 100_000 * 40.0)
    assert abs(w.sum() / 4e6 - 1) < 1e-9
    assert abs(w[0] - np.sqrt(w.sum())) / w[0] < 1e-6
    assert (np.diff(w) <= 0).all()
    # power law: w_i ~ (i + i0)^(-1/1.1) far from the head
    i = np.array([10_000, 90_000])
    slope = np.log(w[i[1]] / w[i[0]]) / np.log(i[1] / i[0])
    assert abs(slope + 1 / 1.1) < 0.05


def test_sbm_shapes_ranges():
    sizes, blocks = graphgen.sbm_shapes(4096, 4)
    assert sizes.min() >= 50 and sizes.max() <= 5000
    assert blocks.min() >= 2 and blocks.max() <= 40
    assert 350 < np.exp(np.log(sizes).mean()) < 700


def _digest(g):
    h = hashlib.sha256()
    h.update(g.off.tobytes())
    h.update(g.col.tobytes())
    return h.hexdigest()


def test_independent_of_thread_count():
    code = ("import sys; sys.path.insert(0, %r); import graphgen, hashlib;"
            "g = graphgen.rmat(13, 16, 0.57, 0.19, 0.19, 9); c = graphgen.chung_lu(20000, 2.1, 12.0, 9);"
            "print(hashlib.sha256(g.off.tobytes() + g.col.tobytes() + c.col.tobytes()).hexdigest())" % ROOT)
    outs = []
    for t in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, check=True,
                                   capture_output=True, text=True).stdout.strip())
    assert outs[0] == outs[1]


def test_seed_changes_graph():
    assert _digest(graphgen.erdos_renyi(1000, 5.0, 1)) != _digest(graphgen.erdos_renyi(1000, 5.0, 2))
