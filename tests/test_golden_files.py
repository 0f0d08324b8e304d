"""The stored end-to-end and gradient references under tests/golden/ against
the seeded inputs and the oracle's readout (CPU only).

The GPU end-to-end tests compare whole solves with these files, so here each
file is checked to still describe the workload its generator names: the
regenerated unary matches its digest, the case parameters match the
generator's case list, and the stored labels and margins are the oracle's
Eq. 3 readout (MAP label, lowest on ties; top-two margin) of the stored
beliefs at every sampled pixel.
"""
import hashlib
import importlib.util
import json
import os

import numpy as np
import pytest

from oracle import grid_bp as gb

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
E2E = sorted(f[4:-4] for f in os.listdir(GOLDEN) if f.startswith("e2e_") and f.endswith(".npz"))


def _generator():
    spec = importlib.util.spec_from_file_location("make_e2e_ref", os.path.join(GOLDEN, "make_e2e_ref.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_generator_uses_the_oracle_only():
    """Stored expected values come from the oracle alone: the generator
    imports nothing of the HIP package."""
    src = open(os.path.join(GOLDEN, "make_e2e_ref.py")).read()
    assert "paper_1010_0012_amd" not in src
    assert "from oracle import" in src


def test_every_case_is_stored():
    gen = _generator()
    assert sorted(gen.case_list()) == E2E


@pytest.mark.parametrize("name", E2E)
def test_e2e_reference(name):
    gen = _generator()
    z = np.load(os.path.join(GOLDEN, f"e2e_{name}.npz"))
    meta = json.loads(str(z["meta"]))
    src, M, T, alpha, mode, sched, n, want_store = gen.case_list()[name]
    assert (meta["source"], meta["M"], meta["T"], meta["mode"], meta["schedule"], meta["n"]) == (
        src, M, T, mode, sched, n)
    assert meta["alpha_f32"] == float(np.float32(alpha))
    g32 = gen.unary(src)
    H, W, _ = g32.shape
    assert (meta["H"], meta["W"]) == (H, W) and g32.shape[2] == M
    assert _digest(g32) == meta["unary_sha256"]

    idx = z["sample_idx"]
    assert idx.dtype == np.int32 and len(np.unique(idx)) == len(idx) == gen.N_SAMPLE
    assert idx.min() >= 0 and idx.max() < H * W
    # the corners are always sampled
    assert {0, W - 1, (H - 1) * W, H * W - 1} <= set(idx.tolist())
    prefixes = [""] + (["store_"] if "store_max_db" in meta else [])
    for p in prefixes:
        b = z[f"{p}sample_b"].astype(np.float64)
        labels, low_idx, low_margin = z[f"{p}labels"], z[f"{p}low_idx"], z[f"{p}low_margin"]
        assert labels.shape == (H, W) and labels.dtype == np.uint8 and labels.max() < M
        assert b.shape == (gen.N_SAMPLE, M) and np.all(b >= 0)
        np.testing.assert_allclose(b.sum(axis=1), 1.0, rtol=0, atol=1e-6 if p else 1e-12)
        # the stored labels are the readout of the stored beliefs (float32
        # rounding of the storage sample can only blur near-ties)
        margin = gb.top2_margin(b.reshape(-1, 1, M)).reshape(-1)
        lab = gb.map_labels(b.reshape(-1, 1, M)).reshape(-1)
        sure = margin > (1e-6 if p else 0.0)
        np.testing.assert_array_equal(lab[sure], labels.reshape(-1)[idx][sure])
        # low_idx lists exactly the pixels whose margin is at most 1e-4
        assert np.all(np.diff(low_idx) > 0) and np.all(low_margin <= gen.LOW_MARGIN)
        in_low = np.isin(idx, low_idx)
        assert np.all(margin[~in_low] > gen.LOW_MARGIN - (1e-6 if p else 0.0))
        pos = np.searchsorted(low_idx, idx[in_low])
        np.testing.assert_allclose(low_margin[pos], margin[in_low], rtol=0, atol=1e-6 if p else 1e-12)
    if "store_max_db" in meta:
        assert meta["store_max_db"] >= 0 and meta["store_map_mismatch"] >= 0
        # the storage model's drift is a property of the whole grid; at the
        # sample (which holds its 512 largest drifts) it is reached
        drift = np.max(np.abs(z["store_sample_b"].astype(np.float64) - z["sample_b"]))
        assert drift == pytest.approx(meta["store_max_db"], rel=1e-3, abs=1e-7)
    assert meta["min_margin"] == pytest.approx(float(z["low_margin"].min()) if len(z["low_idx"]) else
                                               meta["min_margin"])


def test_grad_reference():
    from synth_mrf import CONFIGS, make_config
    z = np.load(os.path.join(GOLDEN, "grad_stereo256grad.npz"))
    meta = json.loads(str(z["meta"]))
    cfg = CONFIGS["stereo256grad"]
    g32, _ = make_config(cfg)
    assert (meta["H"], meta["W"], meta["M"], meta["T"], meta["n"]) == (cfg.H, cfg.W, cfg.M, cfg.T, cfg.iters)
    assert _digest(g32) == meta["unary_sha256"]
    assert z["sample_dtheta"].shape == (len(z["sample_idx"]), cfg.M)
    assert np.max(np.abs(z["sample_dtheta"])) <= meta["max_abs_dtheta"]
    assert np.isfinite(meta["loss"]) and np.isfinite(meta["dalpha"])
