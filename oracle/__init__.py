"""Python handle on the FP64 CPU oracle (``oracle/qtn_oracle.c``).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The HIP library never calls it and
it never calls the HIP library.

``build()`` compiles the C source with gcc into ``oracle/liboracle.so``;
``lib()`` loads it (building first when it is missing).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qtn_oracle.c")
SO = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fcx-limited-range", "-fPIC", "-shared",
          "-pthread", "-Wall", "-Wextra"]

_lib = None


def build(extra_flags=(), out=SO):
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *extra_flags, SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            build()
        L = ctypes.CDLL(SO)
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        i, d = ctypes.c_int, ctypes.c_double
        L.qtno_last_error.restype = ctypes.c_char_p
        L.qtno_lightcone_size.argtypes = [i, i, ip, i, i, i, ip, ip]
        L.qtno_edge_zz.argtypes = [i, i, ip, i, i, dp, dp, i, i, ip, i, dp, dp, ip]
        L.qtno_edge_order.argtypes = [i, i, ip, i, i, i, ip]
        L.qtno_edge_widths.argtypes = [i, i, ip, i, i, i, ip]
        L.qtno_edge_zz_bruteforce.argtypes = [i, i, ip, i, i, dp, dp, i, dp, dp]
        L.qtno_statevector_zz.argtypes = [i, i, ip, i, dp, dp, dp]
        L.qtno_p1_closed_form.argtypes = [i, i, ip, d, d, dp]
        L.qtno_energy.argtypes = [i, i, ip, i, dp, dp, i, i, ip, i, dp, dp, dp]
        L.qtno_contract_bucket.argtypes = [i, ip, ip, dp, i, ip, i, ip, dp]
        L.qtno_mlp_forward.argtypes = [dp, dp, i, dp]
        L.qtno_mlp_loss_grad.argtypes = [dp, dp, dp, dp, i, dp, dp]
        L.qtno_mlp_adam.argtypes = [dp, dp, dp, dp, i, d, d, d, d]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc != 0:
        raise OracleError(f"oracle error {rc}: {lib().qtno_last_error().decode()}")


def _ints(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.int32).ravel())
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _dbls(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _graph(n, edges):
    e, ep = _ints(edges)
    return int(n), len(e) // 2, e, ep


def lightcone_size(n, edges, edge_id, p, mode=0):
    n, m, e, ep = _graph(n, edges)
    nv, nt = ctypes.c_int(), ctypes.c_int()
    _check(lib().qtno_lightcone_size(n, m, ep, edge_id, p, mode,
                                     ctypes.byref(nv), ctypes.byref(nt)))
    return nv.value, nt.value


def edge_order(n, edges, edge_id, p, mode=0):
    nv, _ = lightcone_size(n, edges, edge_id, p, mode)
    n, m, e, ep = _graph(n, edges)
    out, op = _ints(np.zeros(nv))
    _check(lib().qtno_edge_order(n, m, ep, edge_id, p, mode, op))
    return out


def edge_widths(n, edges, edge_id, p, mode=0):
    """Bucket widths by elimination position (symbolic, no arithmetic)."""
    nv, _ = lightcone_size(n, edges, edge_id, p, mode)
    n, m, e, ep = _graph(n, edges)
    out, op = _ints(np.zeros(nv))
    _check(lib().qtno_edge_widths(n, m, ep, edge_id, p, mode, op))
    return out


def edge_zz(n, edges, edge_id, gamma, beta, mode=0, order=None,
            reverse=False, max_width=0, return_widths=False):
    """e_jk (complex) of one edge by bucket elimination."""
    p = len(gamma)
    nv, _ = lightcone_size(n, edges, edge_id, p, mode)
    n, m, e, ep = _graph(n, edges)
    g, gp = _dbls(gamma)
    b, bp = _dbls(beta)
    if order is not None:
        kind = 2
        o, opp = _ints(order)
        if len(o) != nv:
            raise OracleError("order length differs from the variable count")
    else:
        kind = 1 if reverse else 0
        o, opp = None, None
    widths, wp = _ints(np.zeros(nv))
    re, im = ctypes.c_double(), ctypes.c_double()
    _check(lib().qtno_edge_zz(n, m, ep, edge_id, p, gp, bp, mode, kind, opp,
                              max_width, ctypes.byref(re), ctypes.byref(im), wp))
    z = complex(re.value, im.value)
    return (z, widths) if return_widths else z


def edge_zz_bruteforce(n, edges, edge_id, gamma, beta, mode=0):
    p = len(gamma)
    n, m, e, ep = _graph(n, edges)
    g, gp = _dbls(gamma)
    b, bp = _dbls(beta)
    re, im = ctypes.c_double(), ctypes.c_double()
    _check(lib().qtno_edge_zz_bruteforce(n, m, ep, edge_id, p, gp, bp, mode,
                                         ctypes.byref(re), ctypes.byref(im)))
    return complex(re.value, im.value)


def statevector_zz(n, edges, gamma, beta):
    p = len(gamma)
    n, m, e, ep = _graph(n, edges)
    g, gp = _dbls(gamma)
    b, bp = _dbls(beta)
    zz, zp = _dbls(np.zeros(m))
    _check(lib().qtno_statevector_zz(n, m, ep, p, gp, bp, zp))
    return zz


def p1_closed_form(n, edges, gamma, beta):
    n, m, e, ep = _graph(n, edges)
    zz, zp = _dbls(np.zeros(m))
    _check(lib().qtno_p1_closed_form(n, m, ep, float(gamma), float(beta), zp))
    return zz


def energy(n, edges, gamma, beta, mode=0, threads=1, edge_list=None):
    """(zz complex per edge, energy) with min-fill orders.  With edge_list,
    only those edges are evaluated and the energy is None."""
    p = len(gamma)
    n, m, e, ep = _graph(n, edges)
    g, gp = _dbls(gamma)
    b, bp = _dbls(beta)
    if edge_list is None:
        k, lp, cnt = None, None, m
    else:
        k, lp = _ints(edge_list)
        cnt = len(k)
    re, rp = _dbls(np.zeros(cnt))
    im, ipp = _dbls(np.zeros(cnt))
    en = ctypes.c_double()
    _check(lib().qtno_energy(n, m, ep, p, gp, bp, mode, threads, lp, cnt, rp,
                             ipp, ctypes.byref(en)))
    return re + 1j * im, (en.value if edge_list is None else None)


def contract_bucket(tensors, sum_vars, out_idx):
    """Plain contraction of caller-given tensors.

    tensors: list of (idx list, complex ndarray of shape (2,)*rank) with
    idx[0] the most significant (numpy C order).  Returns the complex ndarray
    of shape (2,)*len(out_idx), axes in out_idx order."""
    ranks = [len(ix) for ix, _ in tensors]
    r, rp = _ints(ranks)
    idx, ip = _ints([v for ix, _ in tensors for v in ix] or [0])
    flat = np.concatenate([np.asarray(t, dtype=np.complex128).ravel()
                           for _, t in tensors])
    dat = np.ascontiguousarray(np.stack([flat.real, flat.imag], -1).ravel())
    dp = dat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    s, sp = _ints(list(sum_vars) or [0])
    o, op = _ints(list(out_idx) or [0])
    out = np.zeros(2 * (1 << len(out_idx)))
    _check(lib().qtno_contract_bucket(
        len(tensors), rp, ip, dp, len(sum_vars), sp, len(out_idx), op,
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    res = out[0::2] + 1j * out[1::2]
    return res.reshape((2,) * len(out_idx)) if out_idx else res.reshape(())


# ------------------------------------------------------------- cost model

MLP_SHAPE = (16, 64, 64, 4)


def mlp_nparams():
    return lib().qtno_mlp_nparams()


def mlp_forward(params, x):
    p, pp = _dbls(params)
    xx, xp = _dbls(x)
    n = len(xx) // 16
    y, yp = _dbls(np.zeros(n * MLP_SHAPE[3]))
    _check(lib().qtno_mlp_forward(pp, xp, n, yp))
    return y.reshape(n, MLP_SHAPE[3])


def mlp_loss_grad(params, x, t, m):
    p, pp = _dbls(params)
    xx, xp = _dbls(x)
    tt, tp = _dbls(t)
    mm, mp = _dbls(m)
    n = len(xx) // 16
    g, gp = _dbls(np.zeros(len(p)))
    loss = ctypes.c_double()
    _check(lib().qtno_mlp_loss_grad(pp, xp, tp, mp, n, ctypes.byref(loss), gp))
    return loss.value, g


def mlp_adam(params, m1, m2, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step; returns new (params, m1, m2)."""
    p, pp = _dbls(np.array(params, dtype=np.float64))
    a, ap = _dbls(np.array(m1, dtype=np.float64))
    b, bp = _dbls(np.array(m2, dtype=np.float64))
    g, gp = _dbls(grad)
    _check(lib().qtno_mlp_adam(pp, ap, bp, gp, int(t), lr, beta1, beta2, eps))
    return p, a, b
