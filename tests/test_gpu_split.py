"""The two-site split (tdvp_split) against the oracle's per-sector SVD, at
the benchmark's chi = 4096 middle bond of L = 60 (coupled-sector matrices up
to ~735 on the smaller side, so the eigensolver's 256-1024 buckets run) and on
small tensors with prescribed spectra.

Checked: the reduced singular values of every coupled sector (through their
squares, which the Gram-matrix method fixes to ~1e-16 of the largest), the
kept multiplets against the truncation rule applied to the oracle's values,
the canonical condition of the isometry, and that the product of the two
factors rebuilds theta up to exactly the discarded weight."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2606_04771_amd as T
from oracle import reduced as R
import synth
from tests._harness import torch_stream_handle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    c = T.Context(0, stream=torch_stream_handle())
    yield c
    c.close()


def _upload(blocks, keys, offs, total):
    buf = np.zeros(max(total, 1), np.complex128)
    for k, o in zip(keys, offs):
        a = blocks[tuple(int(v) for v in k)]
        buf[o:o + a.size] = a.reshape(-1, order="F")
    return torch.from_numpy(buf).to("cuda")


def _site(mps, k, left, right):
    keys, offs, data = mps.site(k)
    out = {}
    for key, o in zip(keys, offs):
        r, c = left[key[0]][2], right[key[2]][2]
        out[tuple(int(v) for v in key)] = data[o:o + r * c].reshape((r, c), order="F")
    return out


def _check_split(ctx, left, right, blocks, direction, eps, cap, keep_all=False, iso_tol=1e-12):
    bl, br = T.Bond(left), T.Bond(right)
    xk, xo, xt, xd = T.center_layout(bl, br, 2)
    x_d = _upload(blocks, xk, xo, xt)
    torch.cuda.synchronize()
    mps, sv, disc = ctx.split(bl, br, T.Blocks(xk, xo, x_d.data_ptr(), xt), direction, eps_tol=eps,
                              chi_cap=cap, keep_all=keep_all)
    try:
        ref = R.sector_singular_values(blocks, left, right)
        assert set(ref) == set(sv)
        lam_max = max(float(np.max(v ** 2)) for v in ref.values() if v.size)
        werr = max(float(np.max(np.abs(sv[x] ** 2 - ref[x] ** 2))) for x in ref if ref[x].size)
        print(f"  sectors={len(ref)} largest={max(v.size for v in ref.values())} weight err={werr / lam_max:.2e}",
              flush=True)
        assert werr <= 1e-12 * lam_max
        # the kept multiplets are those the rule keeps on the oracle's values
        mid = mps.bond(1)
        if keep_all:
            want = {x: v.size for x, v in ref.items() if v.size}
        else:
            kept, disc_ref = R.truncate_multiplets(ref, eps, cap)
            want = {x: n for x, n in kept.items() if n}
            assert abs(disc - disc_ref) <= 1e-12
        assert {(q, tj): d for q, tj, d in mid} == want
        # canonical factor and reconstruction
        A = _site(mps, 1, left, mid)
        B = _site(mps, 2, mid, right)
        for ix, (q, tj, d) in enumerate(mid):
            if direction > 0:
                G = sum(a.conj().T @ a for (ia, s, jx), a in A.items() if jx == ix)
            else:
                G = sum(b @ b.conj().T for (jx, s, ib), b in B.items() if jx == ix)
            assert np.abs(G - np.eye(d)).max() < iso_tol, np.abs(G - np.eye(d)).max()
        rebuilt = {}
        for (ia, s1, ix), a in A.items():
            for (jx, s2, ib), b in B.items():
                if jx == ix:
                    key = (ia, s1, mid[ix][1], s2, ib)
                    rebuilt[key] = rebuilt.get(key, 0) + a @ b
        nrm2 = sum(float(np.sum(np.abs(v) ** 2)) for v in blocks.values())
        scale = np.sqrt(1.0 - disc)     # kept values were renormalised to the norm of theta
        res2 = sum(float(np.sum(np.abs(blocks[k] - scale * rebuilt.get(k, 0)) ** 2)) for k in blocks)
        print(f"  kept chi={sum(d * (tj + 1) for _, tj, d in mid)} disc={disc:.3e} "
              f"|theta - A.C|^2/|theta|^2={res2 / nrm2:.3e}", flush=True)
        assert abs(res2 / nrm2 - disc) <= 1e-12
        return sv, disc
    finally:
        mps.close()


@pytest.mark.parametrize("solver", ["trd", "library"])
@pytest.mark.parametrize("direction,eps,cap", [(1, 1e-4, 4096), (-1, 1e-4, 4096), (1, 1e-8, 2048)])
def test_split_at_the_chi4096_middle_bond(ctx, direction, eps, cap, solver, monkeypatch):
    """With trd the Gram matrices of 256 and more go through the in-house
    tridiagonal reduction (the default), with library through the batched
    library solver."""
    monkeypatch.setenv("TDVP_EIG_TRD_MIN", "256" if solver == "trd" else "0")
    print(f"split chi=4096 middle bond direction={direction} eps={eps} cap={cap} eigensolver {solver}", flush=True)
    bonds = synth.random_bonds(60, 4096, 0, center=30)
    left, right = bonds[29], bonds[31]
    keys = [tuple(int(v) for v in k) for k in T.center_layout(T.Bond(left), T.Bond(right), 2)[0]]
    blocks = synth.block_data(keys, [(left[k[0]][2], right[k[4]][2]) for k in keys], 5, 21)
    nrm = np.sqrt(sum(float(np.sum(np.abs(v) ** 2)) for v in blocks.values()))
    # a decaying spectrum, as after time evolution: scale each block by its left sector's weight
    blocks = {k: v / nrm * np.exp(-0.25 * abs(left[k[0]][0])) for k, v in blocks.items()}
    _check_split(ctx, left, right, blocks, direction, eps, cap)


def _spread_theta(left, right, lo, seed):
    """Theta whose every coupled sector has singular values spread
    geometrically from 1 down to lo."""
    rng = np.random.default_rng(seed)
    blocks = {}
    for x, (M, rows, cols) in R.sector_matrices({}, left, right).items():
        r = min(M.shape)
        s = lo ** (np.arange(r) / max(r - 1, 1))
        U, _ = np.linalg.qr(rng.standard_normal((M.shape[0], r)) + 1j * rng.standard_normal((M.shape[0], r)))
        V, _ = np.linalg.qr(rng.standard_normal((M.shape[1], r)) + 1j * rng.standard_normal((M.shape[1], r)))
        Mx = (U * s) @ V.conj().T
        ro = np.cumsum([0] + [left[a][2] for a, _ in rows])
        co = np.cumsum([0] + [right[b][2] for _, b in cols])
        for i, (ia, s1) in enumerate(rows):
            for j, (s2, ib) in enumerate(cols):
                blocks[(ia, s1, x[1], s2, ib)] = Mx[ro[i]:ro[i + 1], co[j]:co[j + 1]]
    return blocks


@pytest.mark.parametrize("direction", [1, -1])
def test_split_isometry_with_a_spread_spectrum(ctx, direction):
    """Singular values spread over 1e-5 (squares over 1e-10), truncation at
    1e-10: where the isometry lies on the larger side it is formed from the
    other side's eigenvectors, and must still be orthonormal to 1e-12."""
    print(f"split spread spectrum direction={direction}", flush=True)
    left = synth.sector_profile(300, 31, parity=1)
    right = synth.sector_profile(120, 32, parity=1) if direction > 0 else synth.sector_profile(300, 32, parity=1)
    if direction < 0:
        left = synth.sector_profile(120, 31, parity=1)
    blocks = _spread_theta(left, right, 1e-5, 7)
    _check_split(ctx, left, right, blocks, direction, 1e-10, 10 ** 6)


@pytest.mark.parametrize("trd_min", ["256", "1"])
def test_split_keep_all_is_exact(ctx, trd_min, monkeypatch):
    monkeypatch.setenv("TDVP_EIG_TRD_MIN", trd_min)
    print(f"split keep_all, tridiagonal reduction from n={trd_min}", flush=True)
    left = synth.sector_profile(200, 41, parity=0)
    right = synth.sector_profile(200, 42, parity=0)
    blocks = _spread_theta(left, right, 1e-3, 9)
    _check_split(ctx, left, right, blocks, 1, 0.0, 10 ** 6, keep_all=True)


@pytest.mark.parametrize("trd_min", ["256", "0"])
def test_split_with_gram_matrices_above_1024(ctx, trd_min, monkeypatch):
    """Few large sectors (chi = 3600 profiles over |2S^z|, 2j <= 2): Gram
    sides up to 1288, so the in-house reduction's large variant (more rows
    per thread, more LDS) runs beside the 1024 and 768 buckets; against the
    oracle, and through the library solver for comparison."""
    monkeypatch.setenv("TDVP_EIG_TRD_MIN", trd_min)
    print(f"split with Gram sides up to 1288, tridiagonal reduction from n={trd_min}", flush=True)
    left = synth.sector_profile(3600, 31, parity=1, qmax=2, tjmax=2)
    right = synth.sector_profile(3600, 32, parity=1, qmax=2, tjmax=2)
    blocks = _spread_theta(left, right, 1e-4, 11)
    _check_split(ctx, left, right, blocks, 1, 1e-10, 10 ** 6)


def test_split_rejects_non_finite_theta(ctx):
    print("split with a NaN in theta", flush=True)
    left = synth.sector_profile(60, 43, parity=0)
    right = synth.sector_profile(60, 44, parity=0)
    bl, br = T.Bond(left), T.Bond(right)
    xk, xo, xt, xd = T.center_layout(bl, br, 2)
    x = np.ones(xt, np.complex128)
    x[xt // 3] = np.nan
    x_d = torch.from_numpy(x).to("cuda")
    torch.cuda.synchronize()
    with pytest.raises(T.TdvpError) as e:
        ctx.split(bl, br, T.Blocks(xk, xo, x_d.data_ptr(), xt), 1)
    assert e.value.code == -7
