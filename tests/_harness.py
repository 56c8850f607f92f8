"""Shared test helpers: synthetic reduced tensors in the library's layouts,
numpy executors of the library's exported host plans, and conversions to
the oracle's full tensors.  Test infrastructure only."""
import numpy as np

import synth
from oracle import reduced as R

_STREAM = []


def torch_stream_handle():
    """Handle of one non-default torch stream, made current for the process,
    so that torch's kernels and the library's (launched on the same handle)
    run in issue order.  torch's default stream has the null handle, for
    which the library would create a private non-blocking stream instead.
    Work issued earlier on other streams is finished first."""
    import torch
    if not _STREAM:
        _STREAM.append(torch.cuda.Stream())
    torch.cuda.synchronize()
    torch.cuda.set_stream(_STREAM[0])
    return _STREAM[0].cuda_stream


def bond_from_profile(chi, seed, parity):
    return synth.sector_profile(chi, seed, parity=parity)


def random_blocks(keys, dims, seed, tag=0):
    return synth.block_data([tuple(k) for k in keys], dims, seed, tag)


def keyed(keys, blocks):
    """dict keyed by tuple -> list in key order"""
    return [blocks[tuple(k)] for k in keys]


def exec_heff_plan(terms, xs, Ls, Rs):
    ys = [np.zeros_like(x) for x in xs]
    for kind, out, inn, env, coef in terms:
        if kind == 0:
            ys[out] += coef * (Ls[env] @ xs[inn])
        elif kind == 1:
            ys[out] += coef * (xs[inn] @ Rs[env].T)
        else:
            ys[out] += coef * xs[inn]
    return ys


def exec_env_plan(terms, direction, ts, Es, out_dims):
    outs = [np.zeros(d, complex) for d in out_dims]
    for kind, o, bra, ket, env, coef in terms:
        if direction > 0:
            bra_op, ket_op = ts[bra].conj().T, ts[ket]
        else:
            bra_op, ket_op = ts[bra].conj(), ts[ket].T
        if kind == 0:
            outs[o] += coef * (bra_op @ Es[env] @ ket_op)
        else:
            outs[o] += coef * (bra_op @ ket_op)
    return outs


def theta_dict(keys, arrs):
    return {tuple(int(v) for v in k): a for k, a in zip(keys, arrs)}


def env_dict(keys, arrs):
    return {tuple(int(v) for v in k): a for k, a in zip(keys, arrs)}


def pack(arrs, offsets, total):
    """Concatenate column-major blocks at offsets into one complex vector."""
    buf = np.zeros(total, np.complex128)
    for a, o in zip(arrs, offsets):
        buf[o:o + a.size] = np.asarray(a).reshape(-1, order="F")
    return buf


def unpack(buf, offsets, dims):
    return [np.asarray(buf[o:o + r * c]).reshape((r, c), order="F") for o, (r, c) in zip(offsets, dims)]
