"""GPU tests of the runtime around the kernels: work on a non-default stream,
the workspace release, and the batched autotuner's cache file."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import gen
from gpu_util import assert_labels_equal, oracle_labels, say, to_dev

pytestmark = pytest.mark.gpu
ccmi = pytest.importorskip("paper_1607_06156_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_side_stream_and_workspace_release():
    g = gen.workload("rmat16")
    u, v = to_dev(g.u), to_dev(g.v)
    expect = oracle_labels(g)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())   # the uploads above ran on the default stream
    with torch.cuda.stream(s):
        for route in ("sv", "heuristic", "bfs+sv"):
            say(f"[gpu] side stream {route}")
            lab = ccmi.label(u, v, g.n, route=route)
            assert_labels_equal(lab, expect, f"side stream/{route}")
        b = gen.batch(12, 77, lg_hi=12.0)
        lab_b = ccmi.label_batched(torch.from_numpy(b.u).cuda(), torch.from_numpy(b.v).cuda(),
                                   torch.from_numpy(b.edge_off).cuda(), torch.from_numpy(b.vert_off).cuda())
    s.synchronize()
    parts = [oracle_labels(b.graph(k)) for k in range(b.G)]
    assert np.array_equal(lab_b.cpu().numpy(), np.concatenate(parts))
    # the workspace is released and grown again on the next call
    ccmi.release_workspace()
    assert_labels_equal(ccmi.label(u, v, g.n, route="sv"), expect, "after release")


_TUNE = r"""
import sys
sys.path.insert(0, {root!r})
import torch
import gen
import paper_1607_06156_amd as ccmi
b = gen.batch(32, 4242, lg_hi=13.0)
args = [torch.from_numpy(a).cuda() for a in (b.u, b.v, b.edge_off, b.vert_off)]
lab, st = ccmi.label_batched(*args, stats=True)
print("shape", st["blocks"], st["max_link"], flush=True)
"""


def test_autotune_cache_file(tmp_path):
    """With CC_AUTOTUNE_CACHE set, the first process writes the tuned launch
    shape of the size class there; a second process reads it back and uses it."""
    path = tmp_path / "tune.txt"
    env = dict(os.environ, CC_AUTOTUNE_CACHE=str(path))
    code = _TUNE.format(root=ROOT)
    shapes = []
    for i in range(2):
        say(f"[gpu] autotune cache, process {i}")
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        shapes.append([ln for ln in r.stdout.splitlines() if ln.startswith("shape")][-1])
        lines = [ln for ln in path.read_text().splitlines() if ln.strip()]
        assert len(lines) == 1
        key, blocks, link = lines[0].split()
        assert "/batched/" in key and int(blocks) >= 8 and int(blocks) % 8 == 0 and int(link) >= 1
        assert shapes[-1] == f"shape {blocks} {link}"
    assert shapes[0] == shapes[1]
