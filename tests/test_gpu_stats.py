"""The message-state check (bp_message_stats): the largest change against
the other message buffer, and the count of non-finite entries, against the
same quantities formed on the host from bp_get_messages."""
import numpy as np
import pytest

from bp_gpu_util import say
from synth_mrf import random_unary

pytestmark = pytest.mark.gpu


def grid_for(H, W, M, T, seed):
    import torch
    from paper_1010_0012_amd.grid import Grid
    grid = Grid(H, W)
    grid.set_potential(M, T, 0.6)
    grid.set_unary(torch.from_numpy(random_unary(H, W, M, seed)).cuda())
    return grid


@pytest.mark.parametrize("fuse,H,W,M", [(False, 23, 31, 16), (True, 23, 31, 16), (True, 64, 96, 64),
                                        (False, 9, 7, 5)])
def test_change_against_the_previous_state(fuse, H, W, M):
    """After n iterations the other buffer holds the state the last launch
    read: n - 1 for one-iteration launches, n - 2 for two-iteration ones."""
    grid = grid_for(H, W, M, 2, 40 + M)
    grid.set_sync_fusion(fuse)
    back = 2 if fuse else 1
    grid.iterate("sum", 8 - back)
    before = grid.get_messages().cpu().numpy()
    grid.iterate("sum", back)
    now = grid.get_messages().cpu().numpy()
    change, bad = grid.message_stats()
    want = float(np.max(np.abs(now - before)))
    say(f"{H}x{W} M={M} fuse={fuse}: max change {change:.3e} (host {want:.3e})")
    assert bad == 0
    assert change == want  # the same float32 subtraction
    assert change > 0
    grid.close()


def test_non_finite_entries_are_counted_and_skipped():
    import torch
    grid = grid_for(12, 17, 16, 2, 5)
    grid.set_sync_fusion(False)
    grid.iterate("sum", 3)
    prev = grid.get_messages().cpu().numpy()
    grid.iterate("sum", 1)
    cur = grid.get_messages().cpu().numpy()
    bad_cur = cur.copy()
    flat = bad_cur.reshape(-1)
    idx = np.random.default_rng(3).choice(flat.size, 5, replace=False)
    flat[idx[0]], flat[idx[1]], flat[idx[2]] = np.nan, np.inf, -np.inf
    grid.set_messages(torch.from_numpy(bad_cur).cuda())
    change, bad = grid.message_stats()
    keep = np.isfinite(bad_cur)
    want = float(np.max(np.abs(bad_cur[keep] - prev[keep])))
    assert bad == 3
    assert change == want
    grid.close()


def test_stats_argument_errors():
    from paper_1010_0012_amd import _lib as L
    grid = grid_for(4, 4, 8, 1, 1)
    with pytest.raises(L.BPError) as e:
        L.bp_message_stats(grid.handle, None, None)
    assert e.value.status == L.BP_EINVAL
    grid.close()


def test_roctx_ranges_do_not_change_results():
    """With BP_ROCTX=1 the calls open roctx ranges (looked up at run time);
    a solve in a child process with it set gives the same labels."""
    import os
    import subprocess
    import sys
    code = (
        "import sys, torch, numpy as np\n"
        f"sys.path.insert(0, {os.path.dirname(os.path.dirname(os.path.abspath(__file__)))!r})\n"
        f"sys.path.insert(0, {os.path.dirname(os.path.abspath(__file__))!r})\n"
        "from paper_1010_0012_amd.grid import Grid\n"
        "from synth_mrf import random_unary\n"
        "g = Grid(20, 30); g.set_potential(16, 2, 0.6)\n"
        "g.set_unary(torch.from_numpy(random_unary(20, 30, 16, 9)).cuda())\n"
        "g.iterate('sum', 6); print(''.join(map(str, g.map_labels().cpu().numpy().ravel()[:40])))\n")
    outs = []
    for flag in ("1", "0"):
        env = dict(os.environ, BP_ROCTX=flag)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=100)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(r.stdout.strip().splitlines()[-1])
    assert outs[0] == outs[1]
