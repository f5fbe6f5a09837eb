"""Host-side logic of the benchmark script (no GPU): the node geometry it uses for the per-level
noise study, and its refusal of more than one GPU."""
import os
import subprocess
import sys

import numpy as np

import gen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_node_geometry_matches_the_oracle():
    """Levels, leaf flags and densities equal the oracle's per canonical node; the centre of
    every leaf, from its integer coordinates, is located by the oracle in that same leaf."""
    rng = np.random.default_rng(8)
    tree = gen.random_tree(rng, (3, 2, 4), 3, 0.4)
    level, leaf, rho, coords = bench.node_geometry(tree)
    o = oracle.Model(tree)
    assert np.array_equal(level, o.level_of_nodes())
    assert np.array_equal(leaf, o.leaf_mask)
    assert np.array_equal(rho, o.node_rho())
    ids = np.flatnonzero(leaf)
    centre = (coords[ids] + 0.5) * (2.0 ** -level[ids].astype(np.float64))[:, None]
    lev, node = o.locate(centre)
    assert np.array_equal(node, ids) and np.array_equal(lev, level[ids])


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout
