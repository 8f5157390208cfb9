"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances (per edge |delta e_jk| and |Im e_jk|, and |delta E| / |E|):
complex128 1e-10, complex64 and mixed 1e-5.  Every e_jk is bounded by ||Z_j Z_k|| = 1,
so the per-edge bound is relative to the operator scale.
"""
import json
import math
import os

import numpy as np
import pytest

import qaoa_synth as qs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {0: 1e-10, 1: 1e-5, 2: 1e-5}


def _check(zz, zi, en, ref_zz, ref_en, prec, what=""):
    tol = TOL[prec]
    ref_zz = np.asarray(ref_zz).real
    err = np.max(np.abs(zz - ref_zz))
    assert err <= tol, f"{what}: max |delta e| = {err:.3e} > {tol}"
    if zi is not None:
        assert np.max(np.abs(zi)) <= tol, f"{what}: |Im e| = {np.max(np.abs(zi)):.3e}"
    rel = abs(en - ref_en) / max(abs(ref_en), 1e-300)
    assert rel <= tol, f"{what}: relative energy error {rel:.3e}"


def _run(qtn, n, edges, g, b, prec, **cfg):
    net = qtn.Network(n, edges, g, b, **cfg)
    net.plan(prec)
    zz, zi, en = net.contract()
    net.close()
    return zz, zi, en


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("levels", [1, 8])
def test_cfg1_n10_p1(qtn, orc, gpu, prec, levels):
    for seed in range(10):
        inst = qs.instance(10, 3, 1, seed)
        g, b = inst["angles"][0]
        sv = orc.statevector_zz(10, inst["edges"], g, b)
        ref_en = len(inst["edges"]) / 2 - 0.5 * np.sum(sv)
        print(f"cfg1 seed={seed} prec={prec} levels={levels}", flush=True)
        zz, zi, en = _run(qtn, 10, inst["edges"], g, b, prec, max_levels=levels)
        _check(zz, zi, en, sv, ref_en, prec, f"seed {seed}")


def test_petersen_p1_optimum(qtn, gpu):
    e = qs.petersen_graph()
    g, b = math.atan(1 / math.sqrt(2)), math.pi / 8
    zz, zi, en = _run(qtn, 10, e, [g], [b], 0)
    assert np.max(np.abs((1 - zz) / 2 - (0.5 + 1 / (3 * math.sqrt(3))))) < 1e-12
    assert abs(en / 15 - (0.5 + 1 / (3 * math.sqrt(3)))) < 1e-12


@pytest.mark.parametrize("n,p", [(12, 2), (16, 3), (16, 4), (20, 3)])
@pytest.mark.parametrize("prec", [0, 1])
def test_small_graphs_all_configs(qtn, orc, gpu, n, p, prec):
    inst = qs.instance(n, 3, p, 7)
    g, b = inst["angles"][0]
    ref, ref_en = orc.energy(n, inst["edges"], g, b, threads=8)
    for cfg in [dict(max_levels=1), dict(max_levels=3), dict(max_levels=8),
                dict(small_width=4), dict(small_width=20), dict(eager=True),
                dict(n_streams=1), dict(variant=1), dict(variant=1, small_width=4),
                dict(small_width=4, lane_sum_bits=1), dict(small_width=4, lane_sum_bits=3),
                dict(small_width=4, lane_sum_bits=5), dict(small_width=4, max_levels=2),
                dict(order_trials=8), dict(small_width=4, variant=2, lane_sum_bits=4),
                dict(executor=2), dict(executor=2, small_width=4),
                dict(executor=2, max_levels=1, variant=1), dict(executor=3),
                dict(executor=3, n_streams=2, small_width=8), dict(executor=4),
                dict(executor=4, small_width=4), dict(executor=4, max_levels=1, variant=1),
                dict(executor=5, hybrid_width=8), dict(executor=5, hybrid_width=8, small_width=4),
                dict(executor=5, hybrid_width=1)]:
        print(f"n={n} p={p} prec={prec} cfg={cfg}", flush=True)
        zz, zi, en = _run(qtn, n, inst["edges"], g, b, prec, **cfg)
        _check(zz, zi, en, ref, ref_en, prec, str(cfg))


def test_repeat_and_new_angles_replay(qtn, orc, gpu):
    inst = qs.instance(16, 3, 3, 2, 3)
    e = inst["edges"]
    net = qtn.Network(16, e, *inst["angles"][0])
    net.plan(0)
    first = net.contract()
    again = net.contract()
    assert np.array_equal(first[0], again[0]) and first[2] == again[2]
    for g, b in inst["angles"][1:]:
        net.set_angles(g, b)
        ref, ref_en = orc.energy(16, e, g, b, threads=8)
        zz, zi, en = net.contract()
        _check(zz, zi, en, ref, ref_en, 0, "replay with new angles")
    # a fresh workspace forces a new descriptor upload and capture
    ws2 = qtn.workspace(net.ws_bytes)
    zz2, _, _ = net.contract(ws=ws2)
    assert np.array_equal(zz2, zz)
    net.close()


def test_energy_gradient_closed_form_p1(qtn, gpu):
    """p=1 on the Petersen graph (3-regular, triangle-free): e_uv =
    -sin(4b) sin(g) cos(g)^2 for every edge, so E = 15/2 + (15/2) sin(4b)
    sin(g) cos(g)^2 and its derivatives are known in closed form.  The
    central differences of one batched pass match them to the truncation
    error."""
    e = qs.petersen_graph()
    rng = np.random.default_rng(3)
    net = qtn.Network(10, e, [0.3], [0.2])
    net.plan(0)
    for _ in range(4):
        g, b = rng.uniform(0, math.pi), rng.uniform(0, math.pi / 2)
        en, dg, db = net.energy_gradient([g], [b], step=1e-5)
        c, s_, s4, c4 = math.cos(g), math.sin(g), math.sin(4 * b), math.cos(4 * b)
        assert abs(en - (7.5 + 7.5 * s4 * s_ * c * c)) < 1e-12
        assert abs(dg[0] - 7.5 * s4 * c * (c * c - 2 * s_ * s_)) < 1e-7
        assert abs(db[0] - 30.0 * c4 * s_ * c * c) < 1e-7
    with pytest.raises(qtn.QtnError):
        net.energy_gradient([0.3], [0.2], step=0.0)
    net.close()


def test_energy_gradient_matches_oracle_differences(qtn, orc, gpu):
    """p=3: the GPU gradient equals the same central differences of the FP64
    oracle's energies at the shifted angles."""
    inst = qs.instance(14, 3, 3, 8)
    e = inst["edges"]
    g, b = (np.asarray(x) for x in inst["angles"][0])
    net = qtn.Network(14, e, g, b, small_width=4)
    net.plan(0)
    h = 1e-4
    en, dg, db = net.energy_gradient(g, b, step=h)
    _, ref_en = orc.energy(14, e, g, b, threads=8)
    assert abs(en - ref_en) <= 1e-10 * abs(ref_en)
    for l in range(3):
        for which, grad in ((0, dg), (1, db)):
            up = [g.copy(), b.copy()]
            dn = [g.copy(), b.copy()]
            up[which][l] += h
            dn[which][l] -= h
            _, eu = orc.energy(14, e, up[0], up[1], threads=8)
            _, ed = orc.energy(14, e, dn[0], dn[1], threads=8)
            assert abs(grad[l] - (eu - ed) / (2 * h)) < 1e-6, (which, l)
    net.close()


def test_edge_cases(qtn, orc, gpu):
    cases = [
        (2, [(0, 1)], 1), (2, [(0, 1)], 3),                      # single edge
        (5, [(0, 1), (1, 2), (2, 3), (3, 4)], 2),                 # path
        (6, [(0, 1), (0, 2), (0, 3), (0, 4), (0, 5)], 3),         # star
        (6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)], 2), # two triangles
        (7, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)], 2),         # isolated 4,5,6
        (8, qs.instance(8, 3, 5, 1)["edges"], 5),                 # deep p
    ]
    r = qs.Rng(17)
    for n, e, p in cases:
        g = [math.pi * r.uniform() for _ in range(p)]
        b = [0.5 * math.pi * r.uniform() for _ in range(p)]
        sv = orc.statevector_zz(n, e, g, b)
        ref_en = len(e) / 2 - 0.5 * np.sum(sv)
        for prec in (0, 1):
            print(f"edge case n={n} m={len(e)} p={p} prec={prec}", flush=True)
            zz, zi, en = _run(qtn, n, e, g, b, prec)
            _check(zz, zi, en, sv, ref_en, prec, f"n={n} p={p}")


def test_given_orders(qtn, orc, gpu):
    inst = qs.instance(12, 3, 3, 5)
    e = inst["edges"]
    g, b = inst["angles"][0]
    ref, ref_en = orc.energy(12, e, g, b, threads=8)
    net = qtn.Network(12, e, g, b)
    r = qs.Rng(8)
    orders = []
    for eid in range(len(e)):
        o = list(net.order_minfill(eid))
        for _ in range(4):
            i, j = r.below(len(o)), r.below(len(o))
            o[i], o[j] = o[j], o[i]
        orders.append(o)
    net.plan(0, orders=orders)
    zz, zi, en = net.contract()
    _check(zz, zi, en, ref, ref_en, 0, "perturbed orders")
    net.close()


def test_gamma_zero_gives_half_edges(qtn, gpu):
    inst = qs.instance(30, 3, 4, 0)
    _, b = inst["angles"][0]
    zz, zi, en = _run(qtn, 30, inst["edges"], [0.0] * 4, b, 0)
    assert np.max(np.abs(zz)) < 1e-10 and abs(en - 22.5) < 1e-9


def test_batch_matches_single(qtn, orc, gpu):
    insts = qs.batch_instances(3, 4, 10, 24, (2, 3), d=3)
    nets, refs = [], []
    for it in insts:
        g, b = it["angles"][0]
        net = qtn.Network(it["n"], it["edges"], g, b)
        net.plan(1)
        nets.append(net)
        refs.append(orc.energy(it["n"], it["edges"], g, b, threads=8))
    handles = [n.h for n in nets]
    need = qtn.qtn_batch_workspace(handles)
    ws = qtn.workspace(need)
    total = sum(n.m for n in nets)
    zz, en = qtn.qtn_contract_batch(handles, total, ws)
    off = 0
    for net, (rz, re_) in zip(nets, refs):
        _check(zz[off:off + net.m], None, en[nets.index(net)], rz, re_, 1, "batch")
        off += net.m
    for n in nets:
        n.close()


def test_persistent_bounded_wait_reports_error(qtn, gpu):
    """A spin limit of one poll makes the grid barrier give up at once: every
    block exits and the call reports QTN_EDEVICE instead of a result."""
    inst = qs.instance(16, 3, 3, 3)
    g, b = inst["angles"][0]
    net = qtn.Network(16, inst["edges"], g, b, executor=2, spin_limit=1)
    net.plan(0)
    with pytest.raises(qtn.QtnError) as ei:
        net.contract()
    assert ei.value.code == -4 and "barrier" in str(ei.value)
    net.close()
    # the same plan with the default bound succeeds afterwards
    net = qtn.Network(16, inst["edges"], g, b, executor=2)
    net.plan(0)
    zz, zi, en = net.contract()
    assert np.all(np.isfinite(zz))
    net.close()


def test_dataflow_bounded_wait_reports_error(qtn, gpu):
    """A spin limit of one poll makes the first dependency wait give up: every
    block exits and the call reports QTN_EDEVICE instead of a result."""
    inst = qs.instance(16, 3, 3, 3)
    g, b = inst["angles"][0]
    net = qtn.Network(16, inst["edges"], g, b, executor=4, spin_limit=1)
    net.plan(0)
    with pytest.raises(qtn.QtnError) as ei:
        net.contract()
    assert ei.value.code == -4 and "dependency" in str(ei.value)
    net.close()
    net = qtn.Network(16, inst["edges"], g, b, executor=4)
    net.plan(0)
    zz, zi, en = net.contract()
    assert np.all(np.isfinite(zz))
    net.close()


def test_batch_persistent_and_streams_agree(qtn, orc, gpu):
    # N in [12, 40], p in {2, 3}: oracle widths stay at or below 18
    insts = qs.batch_instances(5, 6, 12, 40, (2, 3), d=3)
    refs = []
    for it in insts:
        g, b = it["angles"][0]
        print(f"oracle n={it['n']} p={it['p']}", flush=True)
        refs.append(orc.energy(it["n"], it["edges"], g, b, threads=8))
    for executor in (0, 1, 4, 5):
        nets = []
        for it in insts:
            g, b = it["angles"][0]
            net = qtn.Network(it["n"], it["edges"], g, b, executor=executor, order_trials=4,
                              hybrid_width=12 if executor == 5 else 0)
            net.plan(0)
            nets.append(net)
        print(f"batch executor={executor}", flush=True)
        handles = [n.h for n in nets]
        ws = qtn.workspace(qtn.qtn_batch_workspace(handles))
        zz, en = qtn.qtn_contract_batch(handles, sum(n.m for n in nets), ws)
        off = 0
        for i, (net, (rz, re_)) in enumerate(zip(nets, refs)):
            _check(zz[off:off + net.m], None, en[i], rz, re_, 0, f"batch executor {executor}")
            off += net.m
        for n in nets:
            n.close()


@pytest.mark.parametrize("executor", [0, 5])
def test_batch_autotune_keeps_results(qtn, orc, gpu, executor):
    """The batched call's schedule search (persistent grid of all, three
    quarters or half of the resident blocks; step items costliest cone first
    or reversed) gives bit-identical results in the configuration it keeps,
    and on the oracle's values; the launch executors have no such search."""
    insts = qs.batch_instances(7, 5, 12, 36, (2, 3), d=3)
    nets = []
    for it in insts:
        g, b = it["angles"][0]
        net = qtn.Network(it["n"], it["edges"], g, b, executor=executor, order_trials=4,
                          hybrid_width=12 if executor == 5 else 0)
        net.plan(0)
        nets.append(net)
    handles = [n.h for n in nets]
    total = sum(n.m for n in nets)
    ws = qtn.workspace(qtn.qtn_batch_workspace(handles))
    print(f"batch autotune executor={executor}", flush=True)
    zz0, en0 = qtn.qtn_contract_batch(handles, total, ws)
    rep = qtn.qtn_autotune_batch(handles, ws)
    assert rep["n_candidates"] == 6 and 0 <= rep["pick"] < 6
    assert rep["item_order"] == [0, 0, 0, 1, 1, 1]
    gb = rep["grid_blocks"]
    assert gb[0] == gb[3] and gb[0] >= gb[1] >= gb[2] >= 8
    assert all(g % 8 == 0 for g in gb[1:3]) and all(m > 0 for m in rep["ms"])
    zz1, en1 = qtn.qtn_contract_batch(handles, total, ws)
    assert np.array_equal(zz0, zz1) and np.array_equal(en0, en1)
    off = 0
    for i, (it, net) in enumerate(zip(insts, nets)):
        g, b = it["angles"][0]
        rz, re_ = orc.energy(it["n"], it["edges"], g, b, threads=8)
        _check(zz1[off:off + net.m], None, en1[i], rz, re_, 0, f"tuned batch {executor}")
        off += net.m
    for n in nets:
        n.close()
    # launch executors: no persistent grid to tune
    it = insts[0]
    net = qtn.Network(it["n"], it["edges"], *it["angles"][0], executor=1)
    net.plan(0)
    ws1 = qtn.workspace(qtn.qtn_batch_workspace([net.h]))
    with pytest.raises(qtn.QtnError) as ei:
        qtn.qtn_autotune_batch([net.h], ws1)
    assert "persistent" in str(ei.value)
    net.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_keeps_parity(qtn, orc, gpu, prec):
    inst = qs.instance(20, 3, 3, 4)
    g, b = inst["angles"][0]
    ref, ref_en = orc.energy(20, inst["edges"], g, b, threads=8)
    net = qtn.Network(20, inst["edges"], g, b)
    net.plan(prec)
    rep = net.autotune()
    assert rep["n_candidates"] == 7 and rep["n_groups"] > 0
    # the first four candidates time every group; the matrix form only the
    # groups that have one, the cell mapping (3 and 4 cell bits) the groups
    # wide enough for it
    assert rep["tuned_ms"] <= min(rep["cand_ms"][:4]) * (1 + 1e-9)
    assert rep["cand_ms"][4] >= 0 and rep["cand_ms"][5] > 0
    assert sum(rep["picks"]) == rep["n_groups"]
    feats, ms = net.tune_log()
    assert feats.shape[1] == 16 and len(feats) == len(ms) > 0
    assert np.all(ms[:, 2] > 0)
    zz, zi, en = net.contract()
    _check(zz, zi, en, ref, ref_en, prec, "after autotune")
    net.close()


def test_autotune_on_angle_batches_keeps_parity(qtn, orc, gpu):
    """Tuning on angle batches: every candidate runs over 4 copies of the
    angles; the tuned plan matches the oracle for single calls and batches."""
    inst = qs.instance(20, 3, 3, 6, 3)
    e = inst["edges"]
    gs = np.array([a[0] for a in inst["angles"]])
    bs = np.array([a[1] for a in inst["angles"]])
    net = qtn.Network(20, e, gs[0], bs[0], small_width=8)
    net.plan(0)
    need = qtn.qtn_tune_angles_workspace(net.h, 4)
    assert need >= net.angles_workspace(4) > 0
    with pytest.raises(qtn.QtnError):
        qtn.qtn_autotune_angles(net.h, qtn.workspace(need // 2), 4)
    rep = net.autotune(n_sets=4)
    assert rep["n_candidates"] == 7 and rep["n_groups"] > 0 and rep["n_sets"] == 4
    assert rep["tuned_ms"] <= min(rep["cand_ms"][:4]) * (1 + 1e-9)
    zz, en = net.contract_angles(gs, bs)
    for k in range(3):
        ref, ref_en = orc.energy(20, e, gs[k], bs[k], threads=8)
        _check(zz[k], None, en[k], ref, ref_en, 0, f"batch-tuned set {k}")
        net.set_angles(gs[k], bs[k])
        z1, _, e1 = net.contract()
        assert np.array_equal(z1, zz[k]) and e1 == en[k]
    net.close()


@pytest.mark.parametrize("n,p", [(16, 3), (20, 3)])
def test_mixed_precision(qtn, orc, gpu, n, p):
    """Mixed: groups of union width >= mixed_width in complex64, the rest (and
    every group ending in a scalar) in complex128, converting on load."""
    inst = qs.instance(n, 3, p, 11)
    g, b = inst["angles"][0]
    ref, ref_en = orc.energy(n, inst["edges"], g, b, threads=8)
    for mw in (1, 4, 8, 12):
        for cfg in [dict(), dict(small_width=4), dict(variant=1, small_width=4),
                    dict(variant=2, small_width=4, lane_sum_bits=1), dict(executor=2),
                    dict(executor=2, small_width=4, max_levels=2)]:
            print(f"mixed n={n} p={p} mixed_width={mw} cfg={cfg}", flush=True)
            zz, zi, en = _run(qtn, n, inst["edges"], g, b, 2, mixed_width=mw, **cfg)
            _check(zz, zi, en, ref, ref_en, 2, f"mixed {mw} {cfg}")
    # no group reaches width 32: mixed is then the complex128 path exactly
    full = _run(qtn, n, inst["edges"], g, b, 0, small_width=4)
    same = _run(qtn, n, inst["edges"], g, b, 2, small_width=4, mixed_width=32)
    assert np.array_equal(full[0], same[0]) and full[2] == same[2]


@pytest.mark.parametrize("n,p", [(14, 3), (16, 3), (20, 3)])
def test_matrix_form_parity(qtn, orc, gpu, n, p):
    """Matrix form (3M: three real products per complex product on the matrix
    cores) for every group that has one: complex64 (FP32) in its own launch,
    inside workgroups and in the persistent executors; complex128 (FP64) in
    own launches."""
    inst = qs.instance(n, 3, p, 5)
    g, b = inst["angles"][0]
    ref, ref_en = orc.energy(n, inst["edges"], g, b, threads=8)
    for prec, cfg in [(1, dict(small_width=4)), (1, dict()), (1, dict(small_width=4, max_levels=1)),
                      (1, dict(small_width=4, max_levels=2)), (1, dict(executor=2, small_width=4)),
                      (1, dict(executor=4, small_width=4)),
                      (2, dict(small_width=4, mixed_width=6)), (2, dict(mixed_width=1)),
                      (0, dict()), (0, dict(small_width=4, max_levels=2)),
                      (2, dict(mixed_width=30))]:
        print(f"matrix form n={n} p={p} prec={prec} cfg={cfg}", flush=True)
        net = qtn.Network(n, inst["edges"], g, b, variant=3, **cfg)
        net.plan(prec)
        assert net.stats()["n_matrix"] > 0
        zz, zi, en = net.contract()
        _check(zz, zi, en, ref, ref_en, prec, f"matrix form {cfg}")
        if cfg.get("executor", 0) not in (2, 4):
            net.contract_timed()
            log = net.launch_log()
            if cfg.get("small_width") == 4:
                assert any(r["kind"] == 2 and r["variant"] == 2 for r in log)
        net.close()


@pytest.mark.parametrize("n,p", [(12, 2), (16, 3), (20, 3)])
def test_cell_mapping_parity(qtn, orc, gpu, n, p):
    """Cell mapping (lanes on union bits 0..5, kept bits in registers) for
    every group wide enough for it: own launches, inside workgroups, in the
    persistent executors, at 2 and 3 register bits, across summed-bit counts
    below, at and above the six lane bits, in every precision."""
    inst = qs.instance(n, 3, p, 13)
    g, b = inst["angles"][0]
    ref, ref_en = orc.energy(n, inst["edges"], g, b, threads=8)
    for prec, cfg in [(0, dict(small_width=4)), (0, dict(small_width=4, lane_sum_bits=3)),
                      (0, dict(small_width=4, max_levels=1)), (0, dict(small_width=4, max_levels=6)),
                      (0, dict()), (0, dict(small_width=20, lane_sum_bits=3)),
                      (0, dict(executor=2, small_width=4)), (0, dict(executor=4, small_width=4)),
                      (1, dict(small_width=4)), (1, dict(small_width=4, lane_sum_bits=3)),
                      (2, dict(small_width=4, mixed_width=8)),
                      (2, dict(small_width=4, mixed_width=1, lane_sum_bits=3)),
                      (0, dict(small_width=4, lane_sum_bits=4)), (1, dict(small_width=4, lane_sum_bits=4)),
                      (2, dict(small_width=4, mixed_width=8, lane_sum_bits=4))]:
        print(f"cells n={n} p={p} prec={prec} cfg={cfg}", flush=True)
        net = qtn.Network(n, inst["edges"], g, b, variant=4, **cfg)
        net.plan(prec)
        zz, zi, en = net.contract()
        _check(zz, zi, en, ref, ref_en, prec, f"cells {cfg}")
        n_cell = net.stats()["n_cell"]
        if cfg.get("executor", 0) in (2, 4):
            assert n_cell == 0  # the persistent executors run no cell groups
        if n_cell:
            net.contract_timed()
            assert any(r["kind"] == 2 and r["variant"] == 3 for r in net.launch_log())
        elif cfg.get("small_width") == 4 and cfg.get("executor", 0) == 0:
            assert cfg.get("lane_sum_bits") == 4 and n == 12  # no group wide enough
        net.close()


def test_cell_mapping_angle_batch(qtn, orc, gpu):
    """Cell mapping over an angle batch: each set equals its single-set run."""
    inst = qs.instance(20, 3, 3, 21, 3)
    e = inst["edges"]
    gs = np.array([a[0] for a in inst["angles"]])
    bs = np.array([a[1] for a in inst["angles"]])
    net = qtn.Network(20, e, gs[0], bs[0], variant=4, small_width=4, lane_sum_bits=3)
    net.plan(0)
    zz, en = net.contract_angles(gs, bs)
    for k in range(3):
        net.set_angles(gs[k], bs[k])
        z1, _, e1 = net.contract()
        assert np.array_equal(z1, zz[k]) and e1 == en[k], k
        ref, ref_en = orc.energy(20, e, gs[k], bs[k], threads=8)
        _check(zz[k], None, en[k], ref, ref_en, 0, f"cells set {k}")
    net.close()


def _golden(name):
    with open(os.path.join(HERE, "golden", f"{name}_oracle.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("prec,levels,variant,trials,executor", [
    (0, 8, 0, 0, 0), (1, 8, 0, 0, 0), (0, 1, 0, 0, 0), (0, 8, 1, 0, 0), (1, 1, 0, 0, 0),
    (0, 8, 0, 64, 0), (1, 8, 0, 64, 0), (0, 8, 2, 16, 0), (0, 8, 0, 64, 2), (1, 8, 1, 64, 2),
    (0, 8, 0, 64, 3), (2, 8, 0, 64, 0), (2, 8, 0, 64, 2), (1, 8, 3, 64, 0), (2, 8, 3, 64, 0),
    (0, 8, 0, 64, 4), (1, 8, 3, 64, 4), (0, 8, 4, 64, 0), (1, 8, 4, 64, 0), (2, 8, 4, 64, 0),
    (0, 8, 4, 64, 2), (0, 8, 0, -16, 0), (1, 8, 4, -64, 0), (0, 8, 0, 64, 5), (1, 8, 0, 16, 5)])
def test_cfg2_full_size_against_oracle(qtn, gpu, prec, levels, variant, trials, executor):
    """3-regular N=30, p=4 (Sec. II-E benchmark shape), all 45 light cones."""
    gd = _golden("cfg2")
    print(f"cfg2 prec={prec} levels={levels} variant={variant} trials={trials} "
          f"executor={executor}", flush=True)
    # negative trials: orders picked by the merged plan's flops + 4 x bytes
    zz, zi, en = _run(qtn, gd["n"], gd["edges"], gd["gamma"], gd["beta"], prec,
                      max_levels=levels, variant=variant, order_trials=abs(trials),
                      executor=executor, order_weight=4 if trials < 0 else 0)
    _check(zz, zi, en, gd["zz_re"], gd["energy"], prec, "cfg2")


@pytest.mark.parametrize("prec,variant,mixed_width", [
    (0, 0, 0), (1, 0, 0), (2, 0, 18), (2, 3, 18), (1, 3, 0), (2, 3, 12), (0, 4, 0), (2, 4, 18)])
def test_cfg4_full_size_against_oracle(qtn, gpu, prec, variant, mixed_width):
    """4-regular N=40, p=3, all 80 light cones; mixed precision runs groups of
    width >= mixed_width in complex64 (matrix form where it applies with
    variant 3) and reports the per-edge error against the FP64 oracle."""
    gd = _golden("cfg4")
    print(f"cfg4 prec={prec} variant={variant} mixed_width={mixed_width}", flush=True)
    zz, zi, en = _run(qtn, gd["n"], gd["edges"], gd["gamma"], gd["beta"], prec,
                      variant=variant, order_trials=16, mixed_width=mixed_width)
    err = np.abs(zz - np.asarray(gd["zz_re"]))
    print(f"  per-edge |delta e|: max {err.max():.3e} median {np.median(err):.3e}; "
          f"|delta E|/E {abs(en - gd['energy']) / gd['energy']:.3e}", flush=True)
    _check(zz, zi, en, gd["zz_re"], gd["energy"], prec, "cfg4")


@pytest.mark.parametrize("prec", [0, 2])
def test_cfg4_sliced_against_oracle(qtn, gpu, prec):
    """4-regular N=40, p=3 with the headline's plan options: best of 64 orders
    by plan flops + 4 x bytes, light cones wider than 26 sliced (their slices'
    scalars summed in FP64), tuned; per edge against the unsliced FP64 oracle
    values."""
    gd = _golden("cfg4")
    net = qtn.Network(gd["n"], gd["edges"], gd["gamma"], gd["beta"], order_trials=64,
                      slice_width=26, order_weight=4)
    net.plan(prec)
    st = net.stats()
    print(f"cfg4 sliced at 26, prec={prec}: max width {st['max_width']}, "
          f"{st['n_sliced']} cones sliced", flush=True)
    assert st["max_width"] <= 26 and st["n_sliced"] > 0
    net.autotune()
    zz, zi, en = net.contract()
    _check(zz, zi, en, gd["zz_re"], gd["energy"], prec, "cfg4 sliced")
    net.close()


def test_stored_tuning_reapplies(qtn, orc, gpu):
    """Choices measured on one network reapplied to a fresh plan of the same
    graph give the same schedule and results."""
    inst = qs.instance(20, 3, 3, 6)
    g, b = inst["angles"][0]
    ref, ref_en = orc.energy(20, inst["edges"], g, b, threads=8)
    a = qtn.Network(20, inst["edges"], g, b, order_trials=4)
    a.plan(1)
    a.autotune()
    picks = a.tune_picks()
    za, _, ea = a.contract()
    a.contract_timed()
    log_a = [(r["kind"], r["group"], r["variant"]) for r in a.launch_log()]
    bnet = qtn.Network(20, inst["edges"], g, b, order_trials=4)
    bnet.plan(1)
    bnet.set_tune_picks(picks)
    zb, _, eb = bnet.contract()
    bnet.contract_timed()
    log_b = [(r["kind"], r["group"], r["variant"]) for r in bnet.launch_log()]
    assert log_a == log_b
    assert np.array_equal(za, zb) and ea == eb
    _check(zb, None, eb, ref, ref_en, 1, "stored tuning")
    a.close()
    bnet.close()


@pytest.mark.parametrize("prec,cfg", [
    (0, dict()), (0, dict(small_width=4)), (0, dict(small_width=4, variant=2, lane_sum_bits=1)),
    (1, dict(small_width=4, variant=3)), (2, dict(small_width=4, mixed_width=8)),
    (0, dict(executor=3, small_width=8)), (0, dict(executor=2)), (0, dict(eager=True))])
def test_angle_batch_matches_single_sets(qtn, orc, gpu, prec, cfg):
    """Several angle sets in one pass: every set equals its own single-set
    evaluation bit for bit, and the oracle to the tolerance."""
    inst = qs.instance(16, 3, 3, 9, 5)
    e = inst["edges"]
    gs = np.array([a[0] for a in inst["angles"]])
    bs = np.array([a[1] for a in inst["angles"]])
    net = qtn.Network(16, e, gs[0], bs[0], **cfg)
    net.plan(prec)
    print(f"angle batch prec={prec} cfg={cfg}", flush=True)
    zz, en = net.contract_angles(gs, bs)
    assert zz.shape == (5, len(e)) and en.shape == (5,)
    for k in range(5):
        net.set_angles(gs[k], bs[k])
        z1, _, e1 = net.contract()
        assert np.array_equal(z1, zz[k]) and e1 == en[k], k
        ref, ref_en = orc.energy(16, e, gs[k], bs[k], threads=8)
        _check(zz[k], None, en[k], ref, ref_en, prec, f"set {k}")
    # a different set count reuses the plan with a new layout
    zz2, en2 = net.contract_angles(gs[:2], bs[:2])
    assert np.array_equal(zz2, zz[:2]) and np.array_equal(en2, en[:2])
    net.close()


@pytest.mark.parametrize("n_sets", [1, 33, 1024])
def test_angle_batch_set_counts(qtn, orc, gpu, n_sets):
    """One set, a count past a power of two, and the largest count accepted
    (1024), with the cell mapping forced on the wide groups: sampled sets
    equal their single-set evaluation bit for bit, and the oracle."""
    inst = qs.instance(12, 3, 2, 21, n_sets)
    e = inst["edges"]
    gs = np.array([a[0] for a in inst["angles"]])
    bs = np.array([a[1] for a in inst["angles"]])
    net = qtn.Network(12, e, gs[0], bs[0], small_width=4, variant=4)
    net.plan(0)
    assert net.stats()["n_cell"] > 0
    print(f"angle batch n_sets={n_sets}", flush=True)
    zz, en = net.contract_angles(gs, bs)
    assert zz.shape == (n_sets, len(e)) and en.shape == (n_sets,)
    for k in sorted({0, n_sets // 2, n_sets - 1}):
        net.set_angles(gs[k], bs[k])
        z1, _, e1 = net.contract()
        assert np.array_equal(z1, zz[k]) and e1 == en[k], k
    k = n_sets - 1
    ref, ref_en = orc.energy(12, e, gs[k], bs[k], threads=8)
    _check(zz[k], None, en[k], ref, ref_en, 0, f"set {k} of {n_sets}")
    net.close()


def test_angle_batch_full_size(qtn, gpu):
    """N=30 p=4 with the stored oracle angles as one of four sets."""
    gd = _golden("cfg2")
    inst = qs.instance(30, 3, 4, 0, 4)
    gs = np.array([gd["gamma"]] + [a[0] for a in inst["angles"][1:]])
    bs = np.array([gd["beta"]] + [a[1] for a in inst["angles"][1:]])
    net = qtn.Network(gd["n"], gd["edges"], gd["gamma"], gd["beta"], order_trials=16)
    net.plan(0)
    zz, en = net.contract_angles(gs, bs)
    _check(zz[0], None, en[0], gd["zz_re"], gd["energy"], 0, "angle batch set 0")
    for k in range(1, 4):
        net.set_angles(gs[k], bs[k])
        z1, _, e1 = net.contract()
        assert np.array_equal(z1, zz[k]) and e1 == en[k]
    net.close()


def test_angle_batch_timed_launch_log(qtn, gpu):
    """Timed angle batches: one serialized launch per scheduled kernel, bytes
    covering every set."""
    inst = qs.instance(16, 3, 3, 4, 3)
    gs = np.array([a[0] for a in inst["angles"]])
    bs = np.array([a[1] for a in inst["angles"]])
    net = qtn.Network(16, inst["edges"], gs[0], bs[0], small_width=4)
    net.plan(0)
    zz, en, timing = net.contract_angles(gs, bs, timed=True)
    log = net.launch_log()
    assert len(log) > 0 and all(r["ms"] >= 0 for r in log)
    zz1, en1 = net.contract_angles(gs, bs)
    assert np.array_equal(zz, zz1) and np.array_equal(en, en1)
    net.contract_timed()
    single = {k: v["bytes"] for k, v in net.contract_timed()[2].items()}
    for k, v in timing.items():
        assert abs(v["bytes"] - 3 * single[k]) <= 1e-6 * max(1.0, v["bytes"])
    net.close()


@pytest.mark.parametrize("slice_width,weight,tune", [(24, 4, "tune_n30p4_c128_s24_o4.json"),
                                                     (24, 0, "tune_n30p4_c128_s24.json"),
                                                     (0, 0, "tune_n30p4_c128.json")])
def test_headline_plan_against_oracle(qtn, gpu, slice_width, weight, tune):
    """The benchmark's own plans and step: N=30 p=4 graph seed 0, 8 merged
    levels, 4 streams, best-of-64 orders (by the merged plan's flops + 4 x
    bytes for the headline, else by the sum of 2^width), index slicing at
    width 24 (the headline) or none, the stored kernel choices, and one
    32-set angle batch whose set 0 is the stored oracle angle set.  The
    8-summed-index groups run on the cell mapping with 4 cell bits (2 of
    them serial summed bits)."""
    gd = _golden("cfg2")
    inst = qs.instance(30, 3, 4, 0, 32)
    gs = np.array([a[0] for a in inst["angles"]])
    bs = np.array([a[1] for a in inst["angles"]])
    assert np.array_equal(gs[0], gd["gamma"]) and np.array_equal(bs[0], gd["beta"])
    net = qtn.Network(30, inst["edges"], gs[0], bs[0], max_levels=8, n_streams=4,
                      order_trials=64, slice_width=slice_width, order_weight=weight)
    net.plan(qtn.QTN_C128)
    assert (net.stats()["n_sliced"] > 0) == (slice_width > 0)
    root = os.path.dirname(HERE)
    with open(os.path.join(root, "paper_2204_06045_amd", "tuning", tune)) as f:
        net.set_tune_picks(json.load(f)["picks"])
    aws = qtn.workspace(net.angles_workspace(32))
    zz, en = net.contract_angles(gs, bs, aws)
    _check(zz[0], None, en[0], gd["zz_re"], gd["energy"], 0, "headline set 0")
    m = len(inst["edges"])
    assert np.all(np.abs(zz) <= 1 + 1e-12) and np.all((en >= 0) & (en <= m))
    # the timed pass runs the same launches one at a time and gives the same values
    zt, et, _ = net.contract_angles(gs, bs, aws, timed=True)
    assert np.array_equal(zt, zz) and np.array_equal(et, en)
    log = net.launch_log()
    assert any(r["kind"] == 2 and r["variant"] == 3 and r["knob"] == 4 and r["serial"] == 2
               for r in log)
    net.close()


def _batch_golden():
    """The stored FP64 oracle values of the 64-graph batch and the batch's
    instances, regenerated from the same seeds (digest-checked)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden",
                                                  os.path.join(HERE, "golden", "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    gd = _golden("cfg3")
    insts = qs.batch_instances(gd["master_seed"], gd["count"], gd["n_lo"], gd["n_hi"],
                               tuple(gd["depths"]), d=gd["d"])
    for rec in gd["graphs"]:
        assert mg.instance_digest(insts[rec["index"]]) == rec["digest"], rec["index"]
    return gd, insts


@pytest.mark.parametrize("executor", [0, 5])
def test_batch64_full_size_against_oracle(qtn, gpu, executor):
    """The batched workload at full size: 64 cubic graphs (N even in [20,
    200], p in {2, 3, 4}, 10,155 light cones) planned as the benchmark plans
    them (best of 16 orders, complex64, persistent lockstep executor), all
    contracted in one batched call.  Every stored light cone is compared per
    edge, and every graph the oracle evaluated whole by its energy; the
    stored cones cover depths 2, 3 and 4 and a cone of width 30.  Executor 0
    runs every cone in the persistent lockstep launch, executor 5 the cones
    wider than 20 by per-group launches after it; after the batched call's
    schedule search the results are unchanged bit for bit."""
    gd, insts = _batch_golden()
    nets = []
    for it in insts:
        g, b = it["angles"][0]
        net = qtn.Network(it["n"], it["edges"], g, b, order_trials=16, executor=executor)
        net.plan(qtn.QTN_C64)
        nets.append(net)
    handles = [n.h for n in nets]
    total = sum(n.m for n in nets)
    assert total == 10155
    ws = qtn.workspace(qtn.qtn_batch_workspace(handles))
    print(f"batch64 executor {executor}: {total} light cones, workspace "
          f"{ws.numel() / 2**30:.1f} GiB", flush=True)
    zz, en = qtn.qtn_contract_batch(handles, total, ws)
    offs = np.cumsum([0] + [n.m for n in nets])
    widest, depths, n_edges = 0, set(), 0
    for rec in gd["graphs"]:
        i = rec["index"]
        z = zz[offs[i]:offs[i + 1]]
        ids = np.asarray(rec["edge_ids"])
        err = np.max(np.abs(z[ids] - np.asarray(rec["zz_re"])))
        assert err <= TOL[1], f"graph {i}: max |delta e| {err:.3e}"
        if rec["energy"] is not None:
            assert abs(en[i] - rec["energy"]) <= TOL[1] * abs(rec["energy"]), i
        depths.add(rec["p"])
        n_edges += len(ids)
        widest = max(widest, max(max(nets[i].bucket_widths(int(k))) for k in ids))
    print(f"batch64: {n_edges} light cones compared, widest planned bucket {widest}", flush=True)
    assert depths == {2, 3, 4} and widest >= 30
    # the batched call's schedule search (grid, step item order) keeps every
    # result bit for bit in the configuration it keeps
    rep = qtn.qtn_autotune_batch(handles, ws)
    print(f"batch64 schedule search: pick {rep['pick']}, grids {rep['grid_blocks']}", flush=True)
    zz2, en2 = qtn.qtn_contract_batch(handles, total, ws)
    assert np.array_equal(zz, zz2) and np.array_equal(en, en2)
    for n in nets:
        n.close()


@pytest.mark.parametrize("prec,cap,cfg", [
    (0, 24, dict()), (0, 22, dict(order_trials=16)), (1, 24, dict()), (2, 24, dict()),
    (0, 24, dict(executor=2)), (0, 24, dict(executor=4)), (0, 24, dict(variant=4)),
    (0, 20, dict(order_trials=16, n_streams=1))])
def test_cfg2_sliced_against_oracle(qtn, gpu, prec, cap, cfg):
    """Index slicing at full size: N=30 p=4 with every light cone wider than
    the cap contracted slice by slice on one arena, the slices' scalars
    summed in FP64, against the unsliced oracle values."""
    gd = _golden("cfg2")
    print(f"cfg2 sliced prec={prec} cap={cap} cfg={cfg}", flush=True)
    net = qtn.Network(gd["n"], gd["edges"], gd["gamma"], gd["beta"], slice_width=cap, **cfg)
    net.plan(prec)
    st = net.stats()
    assert st["n_sliced"] > 0 and st["max_width"] <= cap
    zz, zi, en = net.contract()
    _check(zz, zi, en, gd["zz_re"], gd["energy"], prec, f"sliced cap {cap} {cfg}")
    if cfg.get("executor", 0) == 0:
        # an angle batch whose set 0 is the stored set matches the single call
        inst = qs.instance(30, 3, 4, 0, 3)
        gs = np.array([gd["gamma"]] + [a[0] for a in inst["angles"][1:]])
        bs = np.array([gd["beta"]] + [a[1] for a in inst["angles"][1:]])
        za, ea = net.contract_angles(gs, bs)
        assert np.array_equal(za[0], zz) and ea[0] == en
    net.close()


@pytest.mark.parametrize("n,p", [(12, 2), (14, 3), (16, 3)])
def test_sliced_small_graphs_all_configs(qtn, orc, gpu, n, p):
    """Aggressive slicing (caps of 6 to 10: up to 10 fixed variables, 1024
    slices per light cone) under every executor and precision."""
    inst = qs.instance(n, 3, p, 19)
    g, b = inst["angles"][0]
    ref, ref_en = orc.energy(n, inst["edges"], g, b, threads=8)
    for prec, cfg in [(0, dict(slice_width=8)), (0, dict(slice_width=7, small_width=4)),
                      (1, dict(slice_width=8)), (2, dict(slice_width=8, mixed_width=4)),
                      (0, dict(slice_width=8, executor=2)), (0, dict(slice_width=7, executor=4)),
                      (0, dict(slice_width=10, variant=1, small_width=4)),
                      (0, dict(slice_width=8, max_levels=1)), (1, dict(slice_width=8, variant=3))]:
        print(f"sliced n={n} p={p} prec={prec} cfg={cfg}", flush=True)
        net = qtn.Network(n, inst["edges"], g, b, **cfg)
        net.plan(prec)
        zz, zi, en = net.contract()
        _check(zz, zi, en, ref, ref_en, prec, f"sliced {cfg}")
        net.close()


def test_hybrid_executor_timed_run(qtn, orc, gpu):
    """The hybrid executor's timed run (launches serialized) gives the same
    results as its graph replay and records a persistent launch and the
    heavy cones' own launches."""
    inst = qs.instance(16, 3, 3, 23)
    g, b = inst["angles"][0]
    ref, ref_en = orc.energy(16, inst["edges"], g, b, threads=8)
    net = qtn.Network(16, inst["edges"], g, b, executor=5, hybrid_width=9)
    net.plan(0)
    zz, zi, en = net.contract()
    _check(zz, zi, en, ref, ref_en, 0, "hybrid")
    zt, et, timing = net.contract_timed()
    assert np.allclose(zt, zz, rtol=0, atol=1e-13) and abs(et - en) < 1e-12
    kinds = {r["kind"] for r in net.launch_log()}
    assert 4 in kinds and 2 in kinds
    net.close()
