"""Per-workload autotuning of the PCG scheduling knobs (four-slot product tile threshold, poll block):
the chosen values come from the candidate set, are applied to the device and cached per workload; the
scenes themselves are not stepped, and the knobs change no result (trajectories bitwise the same)."""
import os

import numpy as np
import pytest

from paper_2503_05020_amd import ipc as G
from paper_2503_05020_amd import scenes as S

pytestmark = pytest.mark.gpu


def _batch(precision):
    scs = [S.soft_cube_drop(cells=3, edge=0.05, height=0.003 + 0.001 * i, seed=i) for i in range(4)]
    return scs, [G.ipc_create_scene(sc, precision=precision) for sc in scs]


@pytest.mark.parametrize("precision", [G.IPC_FP64, G.IPC_MIXED])
def test_autotune_chooses_caches_and_changes_no_result(precision, tmp_path):
    keep = (G.ipc_get_tuning(G.IPC_TUNE_WIDE_TILES), G.ipc_get_tuning(G.IPC_TUNE_POLL_BLOCK))
    cache = str(tmp_path / "tune.txt")
    try:
        # three steps, the tuning, three more steps; then a fresh batch: six steps at the default knobs
        scs, gs = _batch(precision)
        rc, _ = G.ipc_step_batch(gs, 3)
        assert rc == 0
        before = [G.ipc_get_state(g)[0] for g in gs]
        wide, poll, cached = G.ipc_autotune(gs, 2, cache)
        print("tuned", wide, poll, cached, flush=True)
        assert not cached and wide in (-1, 0, 64, 1 << 30) and poll in (-1, 4, 8, 16)
        assert G.ipc_get_tuning(G.IPC_TUNE_WIDE_TILES) == wide and G.ipc_get_tuning(G.IPC_TUNE_POLL_BLOCK) == poll
        # the scenes were not stepped by the tuning
        for g, b in zip(gs, before):
            assert np.array_equal(G.ipc_get_state(g)[0], b)
        rc, _ = G.ipc_step_batch(gs, 3)
        assert rc == 0
        tuned = [G.ipc_get_state(g)[0] for g in gs]
        for g in gs:
            G.ipc_destroy_scene(g)
        with open(cache) as f:
            lines = f.read().splitlines()
        assert len(lines) == 1 and lines[0].split("\t")[1].split()[:2] == [str(wide), str(poll)]
        # the same workload again: from the cache, nothing appended
        G.ipc_set_tuning(G.IPC_TUNE_POLL_BLOCK, 16)
        scs, gs = _batch(precision)
        assert G.ipc_autotune(gs, 2, cache) == (wide, poll, True)
        with open(cache) as f:
            assert len(f.read().splitlines()) == 1
        # default knobs, the same 6 steps: bitwise the tuned run
        G.ipc_set_tuning(G.IPC_TUNE_WIDE_TILES, -1)
        G.ipc_set_tuning(G.IPC_TUNE_POLL_BLOCK, -1)
        rc, _ = G.ipc_step_batch(gs, 6)
        assert rc == 0
        for g, t in zip(gs, tuned):
            assert np.array_equal(G.ipc_get_state(g)[0], t)
        for g in gs:
            G.ipc_destroy_scene(g)
        with pytest.raises(G.IPCError):
            G.ipc_autotune([], 2, cache)
    finally:
        G.ipc_set_tuning(G.IPC_TUNE_WIDE_TILES, keep[0])
        G.ipc_set_tuning(G.IPC_TUNE_POLL_BLOCK, keep[1])
