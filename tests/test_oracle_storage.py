"""Pins of the oracle's float32 storage model (FP64 arithmetic, every stored
message rounded once to float32).

- every stored entry is a float32 value, under every schedule;
- a flat potential (alpha = 0, fbar = 1) sends uniform messages, so after one
  iteration every live entry is float32(1/M) exactly;
- after a step every stored entry is its exact message (recomputed one
  message at a time) rounded to the nearest float32;
- sum-product stays within rounding of the FP64 result (it contracts
  perturbations): a chain after one sweep is the exact marginal to ~1e-7,
  and a stereo grid after 10 iterations is within 1e-6 of FP64.
"""
import numpy as np
import pytest

from oracle import brute
from oracle import grid_bp as gb
from synth_mrf import CONFIGS, make_config, random_unary
from tests.test_oracle_bruteforce import chain_setup, random_sparse_potential

F32 = np.float32


@pytest.mark.parametrize("schedule,n", [(gb.SYNC, 3), (gb.CHECKERBOARD, 4), (gb.SWEEP, 2)])
@pytest.mark.parametrize("mode", [gb.SUM, gb.MAX])
def test_state_is_float32(schedule, n, mode):
    g = random_unary(5, 6, 9, 1).astype(np.float64)
    pot = gb.truncated_linear(9, 2, 0.7)
    st = gb.run(g, pot, mode, n, schedule, storage=F32)
    np.testing.assert_array_equal(st, st.astype(F32).astype(np.float64))


@pytest.mark.parametrize("schedule", [gb.SYNC, gb.SWEEP])
def test_flat_potential_gives_rounded_uniform(schedule):
    M = 7
    g = random_unary(4, 5, M, 2).astype(np.float64)
    pot = gb.truncated_linear(M, 2, 0.0, 1.0)
    st = gb.run(g, pot, gb.SUM, 1, schedule, storage=F32)
    has = gb.has_neighbor(4, 5)
    assert np.all(st[has] == float(F32(1.0 / M)))


@pytest.mark.parametrize("mode", [gb.SUM, gb.MAX])
def test_step_rounds_each_exact_message_once(mode):
    """Every entry the storage model stores after a step is the exact message
    of Eq. 7 / Eq. 11 (recomputed one message at a time by single_update, a
    separate code path from the vectorised step), rounded to the nearest
    float32: within half an ulp of it, and float32-representable.  Rounding
    before the normalisation, rounding h or the window sums, or a narrower
    format all break the half-ulp bound."""
    H, W, M = 4, 5, 8
    g = random_unary(H, W, M, 3).astype(np.float64)
    pot = gb.truncated_linear(M, 2, 0.9)
    s0 = gb.run(g, pot, mode, 2, storage=F32)
    s1 = gb.sync_step(g, s0, pot, mode, storage=F32)
    rounded = 0
    for r in range(H):
        for c in range(W):
            for o in gb.DIRS:
                dr, dc = gb.OFFSETS[o]
                if not (0 <= r + dr < H and 0 <= c + dc < W):
                    continue
                exact = gb.single_update(g, s0, pot, mode, r, c, o)
                got = s1[gb.OPPOSITE[o], r + dr, c + dc]
                assert np.all(got.astype(F32).astype(np.float64) == got)
                half_ulp = np.spacing(np.abs(exact).astype(F32)).astype(np.float64) / 2
                assert np.all(np.abs(got - exact) <= half_ulp)
                rounded += int(np.sum(got != exact))
    assert rounded > 0   # the model did round


def test_chain_sweep_close_to_exact():
    rng = np.random.default_rng(5)
    pot = random_sparse_potential(rng, 5)
    g, P = chain_setup(rng, 6, 5, False, pot)
    st = gb.run(g, pot, gb.SUM, 1, gb.SWEEP, storage=F32)
    b = gb.beliefs(g, st).reshape(6, 5)
    assert np.max(np.abs(b - brute.marginals(P))) <= 5e-7


def test_sum_product_stays_near_fp64():
    cfg = CONFIGS["stereo16"]
    g32, _ = make_config(cfg)
    g = g32.astype(np.float64)
    pot = gb.truncated_linear(cfg.M, cfg.T, cfg.alpha)
    b64 = gb.beliefs(g, gb.run(g, pot, gb.SUM, cfg.iters))
    b32 = gb.beliefs(g, gb.run(g, pot, gb.SUM, cfg.iters, storage=F32))
    assert 0.0 < np.max(np.abs(b32 - b64)) <= 1e-6
