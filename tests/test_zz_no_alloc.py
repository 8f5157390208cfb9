"""The allocation-free single-bucket entry point (qtn_bucket_contract_noalloc,
descriptors in the library's fixed device array) against the workspace entry
point (qtn_bucket_contract) on the same buckets and data: two calls in a row,
the second on a smaller bucket, each bit for bit equal to the workspace
call's output and within the complex128 tolerance of the FP64 oracle."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _fill(b, rng):
    data = torch.zeros(b.info()["data_bytes"], dtype=torch.uint8, device="cuda")
    host = []
    for labels, off in zip(b.operands, b.offsets):
        n = 1 << len(labels)
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        data[off:off + 16 * n].view(torch.complex128).copy_(torch.from_numpy(x))
        host.append(x)
    return data, host


def _out(b, data):
    n = 1 << len(b.out_labels)
    return data[b.out_offset:b.out_offset + 16 * n].view(torch.complex128).cpu().numpy()


def test_noalloc_matches_workspace_entry_point(qtn, orc, gpu):
    from paper_2204_06045_amd import _capi
    lib = _capi.lib()
    rng = np.random.default_rng(77)
    big = qtn.Bucket([list(range(0, 22)), [0, 1, 2, 3] + list(range(22, 28))],
                     list(range(4, 28)))
    small = qtn.Bucket([[0, 1, 2, 3], [0, 4, 5]], [1, 2, 3, 4, 5])
    # a 64 x 64 x 16 matrix product in matrix form (its row, column and
    # summed-index tables travel in the descriptors too)
    mm = qtn.Bucket([[0, 1, 2, 3] + list(range(4, 10)), [0, 1, 2, 3] + list(range(10, 16))],
                    list(range(4, 16)), variant=3)
    assert big.info()["w"] == 28 and small.info()["w"] == 6 and mm.info()["variant"] == 2
    for b in (big, mm, small):  # each call on a smaller input than the one before
        print(f"noalloc bucket w={b.info()['w']} L={b.info()['L']} "
              f"variant={b.info()['variant']}", flush=True)
        data, host = _fill(b, rng)
        rc = lib.qtn_bucket_contract_noalloc(b.h, ctypes.c_void_p(data.data_ptr()),
                                             data.numel(), qtn.stream_handle())
        assert rc == 0, lib.qtn_last_error().decode()
        torch.cuda.synchronize()
        got = _out(b, data).copy()
        data[b.out_offset:].zero_()
        b.contract(data)
        torch.cuda.synchronize()
        assert np.array_equal(got, _out(b, data))
        if b is not big:
            tensors = [(l[::-1], x.reshape((2,) * len(l))) for l, x in zip(b.operands, host)]
            summed = sorted({l for o in b.operands for l in o} - set(b.out_labels))
            ref = np.asarray(orc.contract_bucket(tensors, summed, b.out_labels[::-1])).ravel()
            assert np.max(np.abs(got - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref)))
        else:
            # sampled outputs of the wide bucket against plain sums on the host
            A, B = host
            for o in rng.integers(0, 1 << 24, size=8):
                s = 0
                for k in range(16):
                    ia = k | ((int(o) & ((1 << 18) - 1)) << 4)
                    ib = k | ((int(o) >> 18) << 4)
                    s += A[ia] * B[ib]
                assert abs(got[o] - s) <= 1e-10 * max(1.0, abs(s))
    big.close()
    mm.close()
    small.close()


def test_noalloc_rejects_descriptors_beyond_the_scratch(qtn, gpu):
    # 64 operands on the streaming mapping with 6 serially walked summed
    # labels: their serial-offset tables take the descriptors past 16 KiB
    ops = [list(range(8)) + [8 + k % 16] for k in range(64)]
    b = qtn.Bucket(ops, list(range(8, 24)), variant=2, knob=1)
    info = b.info()
    assert info["variant"] == 1 and info["workspace_bytes"] > 16384
    data = torch.zeros(info["data_bytes"], dtype=torch.uint8, device="cuda")
    with pytest.raises(qtn.QtnError) as ei:
        b.contract_noalloc(data)
    assert ei.value.code == -2 and "scratch" in str(ei.value)
    b.close()
