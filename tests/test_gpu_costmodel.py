"""Learned cost model on the GPU: forward, gradient and Adam against the FP64
oracle; training; the trained selector against the width-rule fallback."""
import math

import numpy as np
import pytest

import qaoa_synth as qs

pytestmark = pytest.mark.gpu


def _rand_params(seed, scale=0.2):
    r = qs.Rng(seed)
    n = 5508
    # uniform in [-scale, scale) from the shared seeded generator
    return np.array([scale * (2 * r.uniform() - 1) for _ in range(n)], dtype=np.float32)


def test_forward_matches_oracle(qtn, orc, gpu):
    p = _rand_params(1)
    r = np.random.default_rng(2)
    x = r.standard_normal((300, 16)).astype(np.float32)
    cm = qtn.CostModel(p)
    y = cm.predict(x)
    ref = orc.mlp_forward(p.astype(np.float64), x.astype(np.float64))
    assert np.max(np.abs(y - ref)) <= 1e-4 * max(1.0, np.max(np.abs(ref)))
    cm.close()


def test_gradient_matches_oracle(qtn, orc, gpu):
    p = _rand_params(3)
    r = np.random.default_rng(4)
    x = r.standard_normal((257, 16)).astype(np.float32)
    t = r.standard_normal((257, 4)).astype(np.float32)
    m = (r.random((257, 4)) > 0.2).astype(np.float32)
    cm = qtn.CostModel(p)
    loss, g = cm.grad(x, t, m)
    rl, rg = orc.mlp_loss_grad(p.astype(np.float64), x.astype(np.float64),
                               t.astype(np.float64), m.astype(np.float64))
    assert abs(loss - rl) <= 1e-4 * max(1.0, rl)
    assert np.max(np.abs(g - rg)) <= 1e-4 * max(1.0, np.max(np.abs(rg)))
    cm.close()


def test_adam_step_matches_oracle(qtn, orc, gpu):
    p = _rand_params(5)
    g = _rand_params(6, scale=1.0)
    cm = qtn.CostModel(p)
    cm.adam_step(g, 0.01)
    cm.adam_step(g * 0.5, 0.01)
    q, m1, m2 = orc.mlp_adam(p.astype(np.float64), np.zeros(len(p)), np.zeros(len(p)),
                             g.astype(np.float64), 1, 0.01)
    q, m1, m2 = orc.mlp_adam(q, m1, m2, (g * 0.5).astype(np.float64), 2, 0.01)
    assert np.max(np.abs(cm.params() - q)) <= 1e-5
    cm.close()


def test_training_reduces_loss(qtn, gpu):
    r = np.random.default_rng(7)
    x = r.uniform(0, 30, (2000, 16)).astype(np.float32)
    # a smooth synthetic timing law: log ms grows with feature 0 and 10
    ms = np.stack([np.exp(0.2 * x[:, 0] - 4), np.exp(0.1 * x[:, 10] - 3),
                   np.exp(0.05 * (x[:, 0] + x[:, 10]) - 3), np.exp(0.15 * x[:, 3] - 5)], 1)
    ms[::5, 0] = -1.0  # unmeasured entries
    ms[::3, 3] = -1.0
    cm = qtn.CostModel(_rand_params(8, 0.1))
    hist = cm.train(x, ms, 400, 3e-3)
    assert hist[-1] < 0.05 * hist[0]
    pred = cm.predict(x[:10])
    assert np.all(np.isfinite(pred))
    cm.close()


def test_costmodel_selection_keeps_parity(qtn, orc, gpu):
    inst = qs.instance(18, 3, 3, 2)
    g, b = inst["angles"][0]
    ref, ref_en = orc.energy(18, inst["edges"], g, b, threads=8)
    net = qtn.Network(18, inst["edges"], g, b)
    net.plan(0)
    net.autotune()
    feats, ms = net.tune_log()
    cm = qtn.CostModel(_rand_params(9, 0.1))
    cm.train(feats, ms, 300, 3e-3)
    counts = qtn.qtn_apply_costmodel(net.h, cm)
    assert counts.sum() == net.stats()["n_groups"]
    zz, zi, en = net.contract()
    assert np.max(np.abs(zz - ref.real)) <= 1e-10
    assert abs(en - ref_en) / abs(ref_en) <= 1e-10
    net.close()
    cm.close()
