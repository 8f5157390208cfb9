"""GPU parity of the single-bucket entry point (qtn_bucket_*, the bucket
kernel alone, Sec. II-B and II-C) against the FP64 oracle's plain bucket
contraction, on seeded random tensors: random label sets, the fixed
abcd,bcdf->acf contraction and matrix products (Sec. II-E) with binary
indices, every kernel mapping, and the degenerate shapes."""
import numpy as np
import pytest
import torch

import qaoa_synth as qs

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-5}


def _device_data(qtn, b, rng, prec):
    """Random operands (seeded) at the bucket's offsets; returns the device
    buffer and the host copies (complex128, rounded to complex64 when the
    bucket is complex64)."""
    es = 8 if prec == qtn.QTN_C64 else 16
    cdt = torch.complex64 if prec == qtn.QTN_C64 else torch.complex128
    data = torch.zeros(max(256, b.info()["data_bytes"]), dtype=torch.uint8, device="cuda")
    host = []
    for labels, off in zip(b.operands, b.offsets):
        n = 1 << len(labels)
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        if prec == qtn.QTN_C64:
            x = x.astype(np.complex64).astype(np.complex128)
        data[off:off + es * n].view(cdt).copy_(torch.from_numpy(x.astype(
            np.complex64 if prec == qtn.QTN_C64 else np.complex128)))
        host.append(x)
    return data, host


def _oracle(orc, b, host):
    """The oracle's bucket contraction: tensors in numpy C order, whose first
    axis is the most significant bit, i.e. the operand's last label."""
    tensors = [(labels[::-1], x.reshape((2,) * len(labels)))
               for labels, x in zip(b.operands, host)]
    summed = sorted({l for o in b.operands for l in o} - set(b.out_labels))
    return np.asarray(orc.contract_bucket(tensors, summed, b.out_labels[::-1])).ravel()


def _run_check(qtn, orc, b, rng, prec, what):
    data, host = _device_data(qtn, b, rng, prec)
    b.contract(data)
    torch.cuda.synchronize()
    es = 8 if prec == qtn.QTN_C64 else 16
    cdt = torch.complex64 if prec == qtn.QTN_C64 else torch.complex128
    n = 1 << len(b.out_labels)
    got = data[b.out_offset:b.out_offset + es * n].view(cdt).cpu().numpy().astype(np.complex128)
    ref = _oracle(orc, b, host)
    err = np.max(np.abs(got - ref))
    scale = max(1.0, np.max(np.abs(ref)))
    assert err <= TOL[prec] * scale, f"{what}: max |delta| {err:.3e} (scale {scale:.3g})"
    return b.info()


def _random_bucket(r, n_ops, n_sum, n_keep, max_rank):
    """Labels 0..n_sum-1 summed, n_sum.. kept; every label held by some
    operand; each operand lists its labels in union order."""
    summed = list(range(n_sum))
    kept = list(range(n_sum, n_sum + n_keep))
    ops = []
    for k in range(n_ops):
        rank = 1 + r.below(max_rank)
        pool = summed + kept
        pick = sorted({pool[r.below(len(pool))] for _ in range(rank)})
        ops.append(pick)
    held = {l for o in ops for l in o}
    for l in summed + kept:
        if l not in held:
            j = r.below(n_ops)
            ops[j] = sorted(set(ops[j]) | {l})
    return ops, kept


@pytest.mark.parametrize("prec", [0, 1])
def test_random_buckets(qtn, orc, gpu, prec):
    r = qs.Rng(606 + prec)
    rng = np.random.default_rng(17 + prec)
    for case in range(24):
        n_ops = 1 + r.below(4)
        n_sum = 1 + r.below(8)
        n_keep = r.below(14)
        ops, kept = _random_bucket(r, n_ops, n_sum, n_keep, 12)
        b = qtn.Bucket(ops, kept, precision=prec)
        info = _run_check(qtn, orc, b, rng, prec, f"case {case}: {ops} -> {kept}")
        print(f"random bucket {case}: w={info['w']} L={info['L']} ops={n_ops} "
              f"variant={info['variant']}", flush=True)
        b.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("variant,knob", [(1, 0), (2, 1), (2, 2), (2, 3), (4, 2), (4, 3),
                                          (4, 4), (3, 0), (0, 0)])
def test_every_mapping(qtn, orc, gpu, prec, variant, knob):
    """Buckets wide enough for every mapping (the union width 14..18, 1..8
    summed labels), each forced onto one mapping; the plan reports the
    mapping it took (a mapping that does not fit falls back to the rule)."""
    r = qs.Rng(900 + 10 * variant + knob)
    rng = np.random.default_rng(variant * 7 + knob)
    taken = set()
    for case in range(6):
        n_sum = 1 + (case * 7) % 8
        n_keep = 14 - n_sum + r.below(4)
        ops, kept = _random_bucket(r, 2 + r.below(3), n_sum, n_keep, 14)
        b = qtn.Bucket(ops, kept, precision=prec, variant=variant, knob=knob)
        info = _run_check(qtn, orc, b, rng, prec, f"variant {variant} knob {knob} case {case}")
        taken.add(info["variant"])
        b.close()
    want = {1: 0, 2: 1, 3: 2, 4: 3}.get(variant)
    if want is not None:
        assert want in taken, (variant, taken)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_fixed_contraction_abcd_bcdf_acf(qtn, orc, gpu, prec, k):
    """abcd,bcdf->acf with every index of size 2^k as k binary labels (the
    fixed expression of the paper's synthetic benchmark); b and d summed."""
    a, bb, c, d, f = ([i * k + j for j in range(k)] for i in range(5))
    # union order: summed labels (b then d) first, then the output a, c, f
    A = bb + d + a + c
    B = bb + d + c + f
    bk = qtn.Bucket([A, B], a + c + f, precision=prec)
    _run_check(qtn, orc, bk, np.random.default_rng(k), prec, f"abcd,bcdf->acf k={k}")
    bk.close()


@pytest.mark.parametrize("prec,variant", [(0, 0), (1, 0), (0, 3), (1, 3)])
@pytest.mark.parametrize("m", [2, 5, 8])
def test_matrix_product(qtn, orc, gpu, prec, variant, m):
    """A 2^m x 2^m matrix product (C[i,j] = sum_k A[i,k] B[k,j]) as a bucket
    with m summed labels (k), m labels of i and m of j."""
    kk = list(range(m))
    ii = list(range(m, 2 * m))
    jj = list(range(2 * m, 3 * m))
    b = qtn.Bucket([kk + ii, kk + jj], ii + jj, precision=prec, variant=variant)
    info = _run_check(qtn, orc, b, np.random.default_rng(m), prec, f"matmul m={m}")
    if variant == 3 and m >= 4:
        assert info["variant"] == 2  # matrix form
    b.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n_sum,n_m,n_n,n_b", [(1, 4, 4, 0), (3, 7, 5, 2), (5, 6, 6, 1),
                                               (8, 9, 4, 0), (6, 4, 8, 3), (2, 12, 7, 0)])
def test_matrix_form_shapes(qtn, orc, gpu, prec, n_sum, n_m, n_n, n_b):
    """Matrix-form buckets: several operands per side, labels shared by both
    sides (batch), an operand with batch and summed labels only, summed
    ranges shorter than and several times one LDS chunk (16), and m / n
    ranges that are not multiples of the 64 x 64 tile.  The operands
    interleave summed and kept labels in union order."""
    r = qs.Rng(4000 + 100 * n_sum + 10 * n_m + n_n)
    labels = list(range(n_sum + n_m + n_n + n_b))
    perm = labels[n_sum:]
    # kept labels shuffled into m / n / batch roles (union positions mixed)
    for i in range(len(perm) - 1, 0, -1):
        j = r.below(i + 1)
        perm[i], perm[j] = perm[j], perm[i]
    mm, nn, bb = perm[:n_m], perm[n_m:n_m + n_n], perm[n_m + n_n:]
    ks = labels[:n_sum]
    a_main = sorted(ks + mm + bb)
    b_main = sorted(ks[: max(1, n_sum - 1)] + nn + bb)
    a_small = sorted(ks[-1:] + mm[:2])
    b_small = sorted(ks[:1] + nn[-3:] + bb[:1])
    ops = [a_main, b_main, a_small, b_small]
    if bb:
        # summed and batch labels only: either side holds it (placed on side B)
        ops.append(sorted(ks[:2] + bb))
    b = qtn.Bucket(ops, sorted(perm), precision=prec, variant=3)
    info = _run_check(qtn, orc, b, np.random.default_rng(n_sum * 31 + n_m), prec,
                      f"matrix form sum={n_sum} m={n_m} n={n_n} b={n_b}")
    print(f"matrix form sum={n_sum} m={n_m} n={n_n} b={n_b}: variant={info['variant']}",
          flush=True)
    assert info["variant"] == 2
    b.close()


def test_degenerate_buckets(qtn, orc, gpu):
    """A full contraction to one scalar, a rank-0 operand, one operand alone,
    repeated operands, and eight summed labels with nothing kept."""
    rng = np.random.default_rng(3)
    for ops, out in [([[0, 1, 2], [0, 1, 2]], []), ([[], [0, 1]], [1]), ([[0, 1, 2, 3]], [2, 3]),
                     ([[0, 3], [0, 3], [0, 3]], [3]), ([list(range(8))], []),
                     ([list(range(8)) + [8, 9], [0, 8]], [8, 9])]:
        for prec in (0, 1):
            b = qtn.Bucket(ops, out, precision=prec)
            _run_check(qtn, orc, b, rng, prec, f"{ops} -> {out}")
            b.close()


def test_bucket_errors_leave_output(qtn, gpu):
    b = qtn.Bucket([[0, 1], [0, 2]], [1, 2])
    small = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(qtn.QtnError) as ei:
        b.contract(small)
    assert ei.value.code == -3  # QTN_ENOMEM
    data = torch.zeros(b.info()["data_bytes"], dtype=torch.uint8, device="cuda")
    with pytest.raises(qtn.QtnError):
        b.contract(data, ws=torch.zeros(16, dtype=torch.uint8, device="cuda"))
    b.close()


def test_timed_run_matches_plain_run(qtn, orc, gpu):
    """The timed entry point runs the same kernel (bit-identical output) and
    reports a positive kernel duration."""
    rng = np.random.default_rng(11)
    b = qtn.Bucket([list(range(18)), [0, 1, 2] + list(range(18, 24))], list(range(3, 24)))
    data, host = _device_data(qtn, b, rng, 0)
    b.contract(data)
    torch.cuda.synchronize()
    n = 1 << len(b.out_labels)
    first = data[b.out_offset:b.out_offset + 16 * n].clone()
    data[b.out_offset:b.out_offset + 16 * n].zero_()
    ms = b.contract_timed(data)
    assert ms > 0
    assert torch.equal(first, data[b.out_offset:b.out_offset + 16 * n])
    b.close()


def test_operand_over_4gib(qtn, orc, gpu):
    """An operand of 8 GiB (rank 29, complex128): the planner routes the
    bucket to the generic mapping (64-bit element offsets) and the output is
    checked on 256 seeded samples, each computed by the oracle's bucket
    contraction from the two input elements it sums.  The inputs are exact
    functions of the element index (residues divided by primes), written on
    the device and recomputed on the host."""
    A = list(range(29))               # label 0 summed, 1..28 kept
    Bk = [0]
    b = qtn.Bucket([A, Bk], list(range(1, 29)), precision=qtn.QTN_C128)
    info = b.info()
    assert info["variant"] == 0       # generic mapping
    na = 1 << 29
    data = torch.empty(info["data_bytes"], dtype=torch.uint8, device="cuda")
    print(f"operand over 4 GiB: data {info['data_bytes'] / 2**30:.1f} GiB", flush=True)

    def fill(off, n):
        view = data[off:off + 16 * n].view(torch.complex128)
        step = 1 << 26
        for s0 in range(0, n, step):
            i = torch.arange(s0, min(n, s0 + step), dtype=torch.float64, device="cuda")
            view[s0:s0 + len(i)] = torch.complex(torch.remainder(i, 1009.0) / 1009.0,
                                                 torch.remainder(i, 997.0) / 997.0 - 0.5)
        return view

    def host(i):
        i = np.asarray(i, dtype=np.float64)
        return np.remainder(i, 1009.0) / 1009.0 + 1j * (np.remainder(i, 997.0) / 997.0 - 0.5)

    fill(b.offsets[0], na)
    wb = np.array([0.75 - 0.25j, -0.5 + 1.0j])
    data[b.offsets[1]:b.offsets[1] + 32].view(torch.complex128).copy_(torch.from_numpy(wb))
    b.contract(data)
    torch.cuda.synchronize()
    out = data[b.out_offset:b.out_offset + 16 * (na // 2)].view(torch.complex128)
    rng = np.random.default_rng(29)
    js = np.concatenate([rng.integers(0, na // 2, 254), [0, na // 2 - 1]])
    got = out[torch.from_numpy(js).to("cuda")].cpu().numpy()
    for j, g in zip(js, got):
        a = host([2 * j, 2 * j + 1])
        ref = np.asarray(orc.contract_bucket([([0], a), ([0], wb)], [0], [])).ravel()[0]
        assert abs(g - ref) <= 1e-12 * max(1.0, abs(ref)), (j, g, ref)
    b.close()
    del data, out
    torch.cuda.empty_cache()
