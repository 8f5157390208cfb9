"""Pins of the FP64 CPU oracle against things other than itself.

- the depth-1 optimum printed in Sec. II-A (0.6924, tests/golden/paper_values.json);
- the published depth-1 closed form (Wang, Hadfield, Jiang, Rieffel 2018);
- a dense matrix exponential of the Hamiltonians of Eq. 1-2 (scipy.linalg.expm);
- numpy.einsum for single-bucket contractions;
- brute-force sums over all variable assignments;
- exact invariants (Sec. II-B energy identity, angle symmetries, MaxCut bound).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import qaoa_synth as qs

HERE = os.path.dirname(os.path.abspath(__file__))


def _paper():
    with open(os.path.join(HERE, "golden", "paper_values.json")) as f:
        return json.load(f)


def test_petersen_p1_optimum_matches_paper(orc):
    pv = _paper()["p1_3regular_ratio"]
    e = qs.petersen_graph()
    zz = orc.statevector_zz(10, e, [pv["gamma"]], [pv["beta"]])
    c_edge = (1 - zz) / 2
    assert np.allclose(c_edge, c_edge[0], atol=1e-14)
    assert abs(c_edge[0] - 0.5 - 1 / (3 * math.sqrt(3))) < 1e-12
    assert 0 <= c_edge[0] - pv["value"] < 1e-4  # printed value, rounded down
    zz_be, energy = orc.energy(10, e, [pv["gamma"]], [pv["beta"]])
    assert np.max(np.abs(zz_be.real - zz)) < 1e-13
    assert abs(energy / len(e) - c_edge[0]) < 1e-13


def _graphs_with_triangles():
    # K4, a triangle with a tail, a 4-regular circulant (has triangles), random cubic
    yield 4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    yield 5, [(0, 1), (1, 2), (0, 2), (2, 3), (3, 4)]
    yield 8, sorted({tuple(sorted((i, (i + s) % 8))) for i in range(8) for s in (1, 2)})
    for seed in range(4):
        yield 10, qs.instance(10, 3, 1, seed)["edges"]


def test_statevector_matches_p1_closed_form(orc):
    r = qs.Rng(99)
    for n, e in _graphs_with_triangles():
        for _ in range(3):
            g, b = math.pi * r.uniform(), 0.5 * math.pi * r.uniform()
            sv = orc.statevector_zz(n, e, [g], [b])
            cf = orc.p1_closed_form(n, e, g, b)
            assert np.max(np.abs(sv - cf)) < 1e-12


def _expm_zz(n, edges, gamma, beta):
    """<Z_j Z_k> from dense exponentials of C (Eq. 1) and B = sum X_i."""
    dim = 1 << n
    z = np.arange(dim)
    bits = (z[:, None] >> np.arange(n)[None, :]) & 1
    cut = sum((bits[:, a] ^ bits[:, b]) for a, b in edges).astype(float)
    C = np.diag(cut)
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    B = np.zeros((dim, dim), dtype=complex)
    for q in range(n):
        op = np.array([[1.0]], dtype=complex)
        for k in reversed(range(n)):
            op = np.kron(op, X if k == q else np.eye(2))
        B += op
    psi = np.full(dim, 1 / math.sqrt(dim), dtype=complex)
    for g, b in zip(gamma, beta):
        psi = scipy.linalg.expm(-1j * g * C) @ psi
        psi = scipy.linalg.expm(-1j * b * B) @ psi
    prob = np.abs(psi) ** 2
    return np.array([np.sum(prob * (1 - 2 * (bits[:, a] ^ bits[:, b]))) for a, b in edges])


def test_statevector_matches_dense_expm(orc):
    r = qs.Rng(5)
    cases = [(4, [(0, 1), (1, 2), (2, 3), (0, 3), (0, 2)]),
             (6, qs.instance(6, 3, 1, 1)["edges"])]
    for n, e in cases:
        for p in (1, 2, 3):
            g = [math.pi * r.uniform() for _ in range(p)]
            b = [0.5 * math.pi * r.uniform() for _ in range(p)]
            ref = _expm_zz(n, e, g, b)
            sv = orc.statevector_zz(n, e, g, b)
            assert np.max(np.abs(sv - ref)) < 1e-12


@pytest.mark.parametrize("n,p", [(6, 1), (8, 2), (10, 1), (10, 2), (10, 3), (12, 2), (12, 4)])
def test_bucket_elimination_matches_statevector(orc, n, p):
    for seed in range(3):
        inst = qs.instance(n, 3, p, 100 + seed)
        e = inst["edges"]
        g, b = inst["angles"][0]
        sv = orc.statevector_zz(n, e, g, b)
        zz, energy = orc.energy(n, e, g, b, threads=4)
        assert np.max(np.abs(zz.real - sv)) < 1e-12
        assert np.max(np.abs(zz.imag)) < 1e-12
        assert abs(energy - (len(e) / 2 - 0.5 * np.sum(sv))) < 1e-11


def test_cfg1_small_instance(orc):
    """N=10 random cubic graphs, p=1: bucket elimination = statevector."""
    for seed in range(10):
        inst = qs.instance(10, 3, 1, seed)
        g, b = inst["angles"][0]
        sv = orc.statevector_zz(10, inst["edges"], g, b)
        zz, _ = orc.energy(10, inst["edges"], g, b, threads=4)
        assert np.max(np.abs(zz.real - sv)) < 1e-12


def test_network_bruteforce_sum(orc):
    inst = qs.instance(12, 3, 1, 3)
    g, b = inst["angles"][0]
    for eid in range(0, len(inst["edges"]), 3):
        nv, _ = orc.lightcone_size(12, inst["edges"], eid, 1)
        assert nv <= 14
        z1 = orc.edge_zz(12, inst["edges"], eid, g, b)
        z2 = orc.edge_zz_bruteforce(12, inst["edges"], eid, g, b)
        assert abs(z1 - z2) < 1e-13
    # a p=2 cone on a small graph (about 20 variables)
    inst = qs.instance(6, 3, 2, 0)
    g, b = inst["angles"][0]
    nv, _ = orc.lightcone_size(6, inst["edges"], 0, 2)
    assert nv <= 24
    z1 = orc.edge_zz(6, inst["edges"], 0, g, b)
    z2 = orc.edge_zz_bruteforce(6, inst["edges"], 0, g, b)
    assert abs(z1 - z2) < 1e-12


def test_order_independence(orc):
    inst = qs.instance(14, 3, 3, 8)
    e = inst["edges"]
    g, b = inst["angles"][0]
    r = qs.Rng(4)
    for eid in (0, 5, 11):
        ref = orc.edge_zz(14, e, eid, g, b)
        rev = orc.edge_zz(14, e, eid, g, b, reverse=True, max_width=30)
        assert abs(ref - rev) < 1e-12
        nv, _ = orc.lightcone_size(14, e, eid, 3)
        mf = list(orc.edge_order(14, e, eid, 3))
        # random swaps of a min-fill order keep widths moderate
        for _ in range(3):
            o = list(mf)
            for _ in range(6):
                i, j = r.below(nv), r.below(nv)
                o[i], o[j] = o[j], o[i]
            z = orc.edge_zz(14, e, eid, g, b, order=o, max_width=30)
            assert abs(ref - z) < 1e-12


def test_lightcone_forms_agree(orc):
    """Reverse light cone = literal subgraph form = whole graph (Sec. II-B)."""
    for n, p, seed in [(8, 1, 0), (8, 2, 1), (10, 2, 2)]:
        inst = qs.instance(n, 3, p, seed)
        e = inst["edges"]
        g, b = inst["angles"][0]
        for eid in range(0, len(e), 4):
            z0 = orc.edge_zz(n, e, eid, g, b, mode=0)
            z1 = orc.edge_zz(n, e, eid, g, b, mode=1)
            z2 = orc.edge_zz(n, e, eid, g, b, mode=2)
            assert abs(z0 - z1) < 1e-12 and abs(z0 - z2) < 1e-12


def _maxcut(n, edges):
    z = np.arange(1 << n)
    bits = (z[:, None] >> np.arange(n)[None, :]) & 1
    return int(max(sum((bits[:, a] ^ bits[:, b]) for a, b in edges)))


def test_energy_invariants(orc):
    n, p = 12, 3
    inst = qs.instance(n, 3, p, 21)
    e = inst["edges"]
    g, b = inst["angles"][0]
    half = len(e) / 2
    _, e0 = orc.energy(n, e, [0.0] * p, b, threads=4)
    _, e1 = orc.energy(n, e, g, [0.0] * p, threads=4)
    assert abs(e0 - half) < 1e-12 and abs(e1 - half) < 1e-12
    zz, en = orc.energy(n, e, g, b, threads=4)
    assert 0 <= en <= _maxcut(n, e) + 1e-12
    assert np.all(np.abs(zz) <= 1 + 1e-12)
    assert abs(en - np.sum((1 - zz.real) / 2)) < 1e-12
    _, en_neg = orc.energy(n, e, [-x for x in g], [-x for x in b], threads=4)
    assert abs(en - en_neg) < 1e-12
    b2 = list(b)
    b2[1] += math.pi / 2
    _, en_b = orc.energy(n, e, g, b2, threads=4)
    assert abs(en - en_b) < 1e-12
    g2 = list(g)
    g2[0] += 2 * math.pi
    _, en_g = orc.energy(n, e, g2, b, threads=4)
    assert abs(en - en_g) < 1e-12


def test_contract_bucket_matches_einsum(orc):
    r = np.random.default_rng(3)
    letters = "abcdefgh"
    for trial in range(6):
        nv = 7
        tensors = []
        for _ in range(3):
            k = r.integers(1, 5)
            idx = sorted(r.choice(nv, size=k, replace=False).tolist())
            data = r.standard_normal((2,) * k) + 1j * r.standard_normal((2,) * k)
            tensors.append((idx, data))
        used = sorted({v for ix, _ in tensors for v in ix})
        n_sum = 1 + trial % 3
        sum_vars = used[:n_sum]
        out_idx = used[n_sum:][::-1]
        got = orc.contract_bucket(tensors, sum_vars, out_idx)
        spec = ",".join("".join(letters[v] for v in ix) for ix, _ in tensors)
        spec += "->" + "".join(letters[v] for v in out_idx)
        ref = np.einsum(spec, *[t for _, t in tensors])
        assert np.max(np.abs(got - ref)) < 1e-12


def test_paper_width27_memory_figure():
    pv = _paper()["width27_c128_bytes"]
    assert abs((1 << 27) * 16 - pv["value"]) / pv["value"] < 0.08


def test_symbolic_widths_match_numeric_run(orc):
    inst = qs.instance(16, 3, 3, 4)
    g, b = inst["angles"][0]
    for eid in range(0, 24, 4):
        _, w = orc.edge_zz(16, inst["edges"], eid, g, b, return_widths=True)
        assert np.array_equal(w, orc.edge_widths(16, inst["edges"], eid, 3))


def test_costmodel_oracle_gradient_by_finite_differences(orc):
    r = np.random.default_rng(11)
    P = orc.mlp_nparams()
    assert P == 16 * 64 + 64 + 64 * 64 + 64 + 64 * 4 + 4
    params = 0.3 * r.standard_normal(P)
    x = r.standard_normal((9, 16))
    t = r.standard_normal((9, 4))
    m = (r.random((9, 4)) > 0.25).astype(float)
    loss, g = orc.mlp_loss_grad(params, x, t, m)
    h = 1e-6
    for q in range(0, P, 53):
        pp = params.copy()
        pp[q] += h
        lp, _ = orc.mlp_loss_grad(pp, x, t, m)
        pp[q] -= 2 * h
        lm, _ = orc.mlp_loss_grad(pp, x, t, m)
        assert abs((lp - lm) / (2 * h) - g[q]) < 1e-6 * max(1.0, abs(g[q]))
    # the loss is the masked mean of squared errors of the forward pass
    y = orc.mlp_forward(params, x)
    assert abs(loss - np.sum(m * (y - t) ** 2) / np.sum(m)) < 1e-12


def test_costmodel_oracle_special_cases(orc):
    P = orc.mlp_nparams()
    # zero weights: the output is the last bias
    params = np.zeros(P)
    params[-4:] = [1.5, -2.0, 0.25, 0.75]
    y = orc.mlp_forward(params, np.ones((4, 16)))
    assert np.allclose(y, [[1.5, -2.0, 0.25, 0.75]] * 4)
    # Adam's first step from zero moments moves every parameter by lr*sign(g)
    g = np.linspace(-1, 1, P)
    g[P // 2] = 0.3
    p1, m1, m2 = orc.mlp_adam(np.zeros(P), np.zeros(P), np.zeros(P), g, 1, 0.01)
    nz = np.abs(g) > 1e-3
    assert np.allclose(p1[nz], -0.01 * np.sign(g[nz]), rtol=1e-4)
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)


def _mlp_numpy_forward(params, x):
    """The 16-64-64-4 perceptron written out with numpy: parameters in the
    order W1[16][64], b1[64], W2[64][64], b2[64], W3[64][4], b3[4]."""
    sizes = [(16, 64), (64,), (64, 64), (64,), (64, 4), (4,)]
    parts, k = [], 0
    for s in sizes:
        n = int(np.prod(s))
        parts.append(np.asarray(params[k:k + n]).reshape(s))
        k += n
    W1, b1, W2, b2, W3, b3 = parts
    h1 = np.maximum(x @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h2 @ W3 + b3


def test_costmodel_oracle_forward_against_numpy(orc):
    # random nonzero weights and biases, negative hidden biases included, so
    # that both hidden ReLUs clip a share of the units
    r = np.random.default_rng(5)
    P = orc.mlp_nparams()
    params = r.standard_normal(P) * 0.4
    params[16 * 64:16 * 64 + 64] -= 0.3          # b1
    params[16 * 64 + 64 + 4096:16 * 64 + 128 + 4096] -= 0.3  # b2
    x = r.standard_normal((37, 16))
    y = orc.mlp_forward(params, x)
    ref = _mlp_numpy_forward(params, x)
    assert np.max(np.abs(y - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))
    # both ReLUs matter on these inputs
    W1 = params[:1024].reshape(16, 64)
    assert np.mean(x @ W1 + params[1024:1088] < 0) > 0.2


def test_costmodel_oracle_forward_hand_case(orc):
    # x = 2 e_0.  Layer 1: units 0, 1 get +2, -2 (unit 1 clipped), unit 2
    # bias -0.5 (clipped), unit 3 bias 0.5.  Layer 2: unit 0 = 3*2 = 6,
    # unit 1 = 1*h1[1] - 4*0.5 = -2 (clipped), unit 2 = 2*0.5 = 1, unit 4 =
    # -1*h1[1] = 0 (2 without the first ReLU).  Output: y0 = 0.5*6 + 0.1,
    # y1 = 1*1 + 0.2, y2 = 7*h2[1] + 0.3 = 0.3 (-13.7 without the second
    # ReLU), y3 = 1*h2[4] + 0.4 = 0.4.
    P = orc.mlp_nparams()
    p = np.zeros(P)
    W1 = np.zeros((16, 64)); b1 = np.zeros(64)
    W2 = np.zeros((64, 64)); b2 = np.zeros(64)
    W3 = np.zeros((64, 4)); b3 = np.array([0.1, 0.2, 0.3, 0.4])
    W1[0, 0], W1[0, 1] = 1.0, -1.0
    b1[2], b1[3] = -0.5, 0.5
    W2[0, 0], W2[1, 1], W2[3, 1], W2[3, 2], W2[1, 4] = 3.0, 1.0, -4.0, 2.0, -1.0
    W3[0, 0], W3[2, 1], W3[1, 2], W3[4, 3] = 0.5, 1.0, 7.0, 1.0
    p[:] = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    x = np.zeros((1, 16)); x[0, 0] = 2.0
    y = orc.mlp_forward(p, x)
    assert np.allclose(y, [[3.1, 1.2, 0.3, 0.4]], atol=1e-15, rtol=0)
