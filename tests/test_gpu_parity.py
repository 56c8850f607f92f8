"""GPU parity of the HIP path against the CPU oracle (FP64 to 1e-12 relative,
FP32 and split-BF16 to 4e-6 relative), through the C ABI, and the error paths
that the host can force without faulting the GPU.

Sizes: bonds with a handful of sectors and degeneracies up to ~80, so blocks
span several 64x64 tiles with ragged tails while the oracle's dense
expansion still finishes in seconds."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2606_04771_amd as T
from oracle import dense as D
from oracle import reduced as R
import synth
from tests._harness import torch_stream_handle, keyed, pack, random_blocks, theta_dict, env_dict, unpack

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
# FP32 accumulation: a few times the sqrt(K) u rounding of the longest chains
# here (K ~ 300 summed products, u = 2^-24): 4 * 17 * 6e-8 ~ 4e-6
FP32_TOL = 4e-6
SPLIT = (0.01, 32)   # K-chain splitting forced down to 32-deep pieces


def _bond(parity, seed, big=80, n_small=3):
    """A few sectors with one big degeneracy (several tiles, ragged tail)."""
    rng = np.random.default_rng(seed)
    labels = [(q, tj) for q in range(-3, 4) for tj in range(0, 4) if (q - tj - parity) % 2 == 0]
    rng.shuffle(labels)
    out = [(labels[0][0], labels[0][1], big + int(rng.integers(0, 9)))]
    for q, tj in labels[1:1 + n_small + 3]:
        out.append((q, tj, int(rng.integers(1, 30))))
    return sorted(out)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    c = T.Context(0, stream=torch_stream_handle())   # ordered with torch's work
    yield c
    c.close()


def dev(buf):
    return torch.from_numpy(buf).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _heff_case(site, nsites, seed):
    lp = (site - 1) % 2
    left = _bond(lp, seed)
    right = _bond(lp if nsites == 2 else 1 - lp, seed + 1)
    bl, br = T.Bond(left), T.Bond(right)
    xk, xo, xt, xd = T.center_layout(bl, br, nsites)
    lk, lo, lt, ld = T.env_layout(bl)
    rk, ro, rt, rd = T.env_layout(br)
    xs = keyed(xk, random_blocks(xk, xd, seed + 2))
    Ls = keyed(lk, random_blocks(lk, ld, seed + 3))
    Rs = keyed(rk, random_blocks(rk, rd, seed + 4))
    return left, right, bl, br, (xk, xo, xt, xd, xs), (lk, lo, lt, ld, Ls), (rk, ro, rt, rd, Rs)


@pytest.mark.parametrize("site,prec,split", [(3, T.FP64, False), (4, T.FP64, False), (3, T.FP32, False),
                                             (3, T.BF16X3, False), (4, T.BF16X3, False), (3, T.FP64, True),
                                             (4, T.FP64, True), (3, T.FP32, True), (4, T.BF16X3, True)])
def test_heff_two_site(ctx, site, prec, split):
    t, U = 1.0, 4.0
    print(f"heff2 site={site} prec={prec} split={split}", flush=True)
    left, right, bl, br, X, Lx, Rx = _heff_case(site, 2, 100 + site)
    xk, xo, xt, xd, xs = X
    lk, lo, lt, ld, Ls = Lx
    rk, ro, rt, rd, Rs = Rx
    x_d = dev(pack(xs, xo, xt))
    y_d = torch.zeros_like(x_d)
    L_d = dev(pack(Ls, lo, lt))
    R_d = dev(pack(Rs, ro, rt))
    model = T.Model(8, t, U)
    ctx.set_precision(prec)
    if split:
        ctx.set_split(*SPLIT)
    try:
        ctx.heff_apply(model, site, 2, bl, br, T.Blocks(lk, lo, L_d.data_ptr(), lt),
                       T.Blocks(rk, ro, R_d.data_ptr(), rt), T.Blocks(xk, xo, x_d.data_ptr(), xt),
                       T.Blocks(xk, xo, y_d.data_ptr(), xt))
        ctx.synchronize()
    finally:
        ctx.set_precision(T.FP64)
        ctx.set_split()
    ys = unpack(host(y_d), xo, xd)
    ref = D.heff2(R.expand_env(env_dict(lk, Ls), left), R.expand_env(env_dict(rk, Rs), right),
                  R.expand_theta(theta_dict(xk, xs), left, right, site), site, t, U)
    got = R.expand_theta(theta_dict(xk, ys), left, right, site)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  max rel err {err:.3e}", flush=True)
    assert err < (FP64_TOL if prec == T.FP64 else FP32_TOL)


def test_heff_one_site(ctx):
    t, U, site = 1.0, 4.0, 5
    left, right, bl, br, X, Lx, Rx = _heff_case(site, 1, 200)
    xk, xo, xt, xd, xs = X
    lk, lo, lt, ld, Ls = Lx
    rk, ro, rt, rd, Rs = Rx
    x_d = dev(pack(xs, xo, xt))
    y_d = torch.zeros_like(x_d)
    L_d = dev(pack(Ls, lo, lt))
    R_d = dev(pack(Rs, ro, rt))
    ctx.heff_apply(T.Model(8, t, U), site, 1, bl, br, T.Blocks(lk, lo, L_d.data_ptr(), lt),
                   T.Blocks(rk, ro, R_d.data_ptr(), rt), T.Blocks(xk, xo, x_d.data_ptr(), xt),
                   T.Blocks(xk, xo, y_d.data_ptr(), xt))
    ys = unpack(host(y_d), xo, xd)
    ref = D.heff1(R.expand_env(env_dict(lk, Ls), left), R.expand_env(env_dict(rk, Rs), right),
                  R.expand_site("C", theta_dict(xk, xs), left, right, site), site, t, U)
    got = R.expand_site("C", theta_dict(xk, ys), left, right, site)
    assert np.abs(got - ref).max() / np.abs(ref).max() < FP64_TOL


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("prec", [T.FP64, T.FP32, T.BF16X3])
@pytest.mark.parametrize("direction", [1, -1])
def test_env_update(ctx, direction, prec, split):
    t, U, site = 1.0, 4.0, 4
    print(f"env update direction={direction} prec={prec} split={split}", flush=True)
    b_site_left = _bond((site - 1) % 2, 300)     # bond site-1
    b_site_right = _bond(site % 2, 301)          # bond site
    if direction > 0:
        bin_, bout = b_site_left, b_site_right
        tk, to, tt, td = T.center_layout(T.Bond(bin_), T.Bond(bout), 1)
    else:
        bin_, bout = b_site_right, b_site_left
        tk, to, tt, td = T.center_layout(T.Bond(bout), T.Bond(bin_), 1)
    bi, bo = T.Bond(bin_), T.Bond(bout)
    ek, eo, et, ed = T.env_layout(bi)
    ok, oo, ot, od = T.env_layout(bo)
    ts = keyed(tk, random_blocks(tk, td, 302))
    Es = keyed(ek, random_blocks(ek, ed, 303))
    t_d = dev(pack(ts, to, tt))
    e_d = dev(pack(Es, eo, et))
    o_d = torch.zeros(max(ot, 1), dtype=torch.complex128, device="cuda")
    ctx.set_precision(prec)
    if split:
        ctx.set_split(*SPLIT)
    try:
        ctx.env_update(T.Model(8, t, U), site, direction, bi, bo, T.Blocks(ek, eo, e_d.data_ptr(), et),
                       T.Blocks(tk, to, t_d.data_ptr(), tt), T.Blocks(ok, oo, o_d.data_ptr(), ot))
        ctx.synchronize()
        outs = unpack(host(o_d), oo, od)
    finally:
        ctx.set_precision(T.FP64)
        ctx.set_split()
    Ef = R.expand_env(env_dict(ek, Es), bin_)
    if direction > 0:
        ref = D.left_env_update(Ef, R.expand_site("A", theta_dict(tk, ts), bin_, bout, site), site, t, U)
    else:
        ref = D.right_env_update(Ef, R.expand_site("B", theta_dict(tk, ts), bout, bin_, site), site, t, U)
    got = R.expand_env(env_dict(ok, outs), bout)
    scale = max(np.abs(ref[w]).max() for w in range(3))
    tol = FP64_TOL if prec == T.FP64 else FP32_TOL
    err = max(np.abs(got[w] - ref[w]).max() for w in range(3)) / scale
    print(f"  max error relative to the largest entry: {err:.2e}", flush=True)
    assert err < tol


def test_heff_deterministic(ctx):
    """FP64 reruns are bit-identical (no atomics, fixed summation order)."""
    left, right, bl, br, X, Lx, Rx = _heff_case(3, 2, 400)
    xk, xo, xt, xd, xs = X
    lk, lo, lt, ld, Ls = Lx
    rk, ro, rt, rd, Rs = Rx
    x_d = dev(pack(xs, xo, xt))
    L_d = dev(pack(Ls, lo, lt))
    R_d = dev(pack(Rs, ro, rt))
    outs = []
    for _ in range(3):
        y_d = torch.full_like(x_d, float("nan"))
        ctx.heff_apply(T.Model(8), 3, 2, bl, br, T.Blocks(lk, lo, L_d.data_ptr(), lt),
                       T.Blocks(rk, ro, R_d.data_ptr(), rt), T.Blocks(xk, xo, x_d.data_ptr(), xt),
                       T.Blocks(xk, xo, y_d.data_ptr(), xt))
        outs.append(host(y_d))
    assert np.isfinite(outs[0]).all()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def _physical_envs(ctx, L, site, nsites, seed, t, U, chi):
    """Reduced MPS (random, mixed-canonical at `site`), environments built on
    the GPU with env_update; returns everything needed for a Krylov test."""
    bonds, sites = synth.random_mps(L, chi, seed, center=site)
    model = T.Model(L, t, U)
    # left environments
    b0 = T.Bond(bonds[0])
    ek, eo, et, ed = T.env_layout(b0)
    env = torch.zeros(max(et, 1), dtype=torch.complex128, device="cuda")
    env_desc = (ek, eo, et, ed)
    keep = []
    for k in range(1, site):
        bi, bo = T.Bond(bonds[k - 1]), T.Bond(bonds[k])
        tk, to, tt, td = T.center_layout(bi, bo, 1)
        t_d = dev(pack(keyed(tk, sites[k - 1]), to, tt))
        ok, oo, ot, od = T.env_layout(bo)
        out = torch.zeros(max(ot, 1), dtype=torch.complex128, device="cuda")
        ctx.env_update(model, k, 1, bi, bo, T.Blocks(env_desc[0], env_desc[1], env.data_ptr(), env_desc[2]),
                       T.Blocks(tk, to, t_d.data_ptr(), tt), T.Blocks(ok, oo, out.data_ptr(), ot))
        keep.append((env, t_d))
        env, env_desc = out, (ok, oo, ot, od)
    Lenv, Ldesc = env, env_desc
    bL = T.Bond(bonds[L])
    ek, eo, et, ed = T.env_layout(bL)
    env = torch.zeros(max(et, 1), dtype=torch.complex128, device="cuda")
    env_desc = (ek, eo, et, ed)
    last = site + nsites - 1
    for k in range(L, last, -1):
        bi, bo = T.Bond(bonds[k]), T.Bond(bonds[k - 1])
        tk, to, tt, td = T.center_layout(bo, bi, 1)
        t_d = dev(pack(keyed(tk, sites[k - 1]), to, tt))
        ok, oo, ot, od = T.env_layout(bo)
        out = torch.zeros(max(ot, 1), dtype=torch.complex128, device="cuda")
        ctx.env_update(model, k, -1, bi, bo, T.Blocks(env_desc[0], env_desc[1], env.data_ptr(), env_desc[2]),
                       T.Blocks(tk, to, t_d.data_ptr(), tt), T.Blocks(ok, oo, out.data_ptr(), ot))
        keep.append((env, t_d))
        env, env_desc = out, (ok, oo, ot, od)
    torch.cuda.synchronize()
    return bonds, sites, model, (Lenv, Ldesc), (env, env_desc)


@pytest.mark.parametrize("nsites,tau,storage", [(2, -0.025j, T.FP64), (1, 0.025j, T.FP64), (2, -0.3j, T.FP64),
                                                (2, -0.3j, T.FP32), (1, 0.025j, T.FP32)])
def test_krylov_expm_against_dense_oracle(ctx, nsites, tau, storage):
    """FP64 basis: 1e-10 of the dense exponential.  Complex64 basis storage
    (FP64 recurrence, rounded basis in the re-orthogonalisation and the final
    combination): a few times the FP32 rounding of the combination, 2e-6."""
    L, site, t, U = 6, 3, 1.0, 4.0
    print(f"krylov nsites={nsites} tau={tau} basis storage {storage}", flush=True)
    bonds, sites, model, (Lenv, Ld), (Renv, Rd) = _physical_envs(ctx, L, site, nsites, 7, t, U, 24)
    left, right = bonds[site - 1], bonds[site + nsites - 1]
    bl, br = T.Bond(left), T.Bond(right)
    xk, xo, xt, xd = T.center_layout(bl, br, nsites)
    xs = keyed(xk, random_blocks(xk, xd, 55))
    nrm = np.sqrt(sum(np.sum(np.abs(a) ** 2) for a in xs))
    xs = [a / nrm for a in xs]
    x_d = dev(pack(xs, xo, xt))
    ctx.set_krylov_storage(storage)
    try:
        rc, info = ctx.krylov_expm(model, site, nsites, bl, br, T.Blocks(Ld[0], Ld[1], Lenv.data_ptr(), Ld[2]),
                                   T.Blocks(Rd[0], Rd[1], Renv.data_ptr(), Rd[2]),
                                   T.Blocks(xk, xo, x_d.data_ptr(), xt), tau, tol=1e-13, maxdim=40)
    finally:
        ctx.set_krylov_storage(T.FP64)
    assert info["converged"], info
    ys = unpack(host(x_d), xo, xd)
    # oracle: dense environments from the expanded MPS, dense exponential
    full = [R.expand_site("A" if k < site else ("C" if k == site else "B"), sites[k - 1], bonds[k - 1],
                          bonds[k], k) for k in range(1, L + 1)]
    Lf = D.empty_env()
    for k in range(1, site):
        Lf = D.left_env_update(Lf, full[k - 1], k, t, U)
    Rf = D.empty_env()
    for k in range(L, site + nsites - 1, -1):
        Rf = D.right_env_update(Rf, full[k - 1], k, t, U)
    if nsites == 2:
        v = R.expand_theta(theta_dict(xk, xs), left, right, site)
        ref, _ = D.lanczos_expm(lambda z: D.heff2(Lf, Rf, z, site, t, U), v, tau, tol=1e-15, maxdim=60)
        got = R.expand_theta(theta_dict(xk, ys), left, right, site)
    else:
        v = R.expand_site("C", theta_dict(xk, xs), left, right, site)
        ref, _ = D.lanczos_expm(lambda z: D.heff1(Lf, Rf, z, site, t, U), v, tau, tol=1e-15, maxdim=60)
        got = R.expand_site("C", theta_dict(xk, ys), left, right, site)
    err = np.abs(got - ref).max()
    print(f"  iters={info['iters']} (graph-replayed {info['graph_iters']}) err={err:.2e}", flush=True)
    if storage == T.FP64:
        assert err < 1e-10
        assert abs(np.linalg.norm(got) - 1.0) < 1e-12
    else:
        assert err < 2e-6
        assert abs(np.linalg.norm(got) - 1.0) < 2e-6


@pytest.mark.parametrize("prec,storage", [(T.FP64, T.FP64), (T.FP32, T.FP64), (T.FP64, T.FP32)])
def test_krylov_graph_replay_matches_direct_launches(ctx, prec, storage):
    """One captured Lanczos iteration replayed for the rest of the exponential
    gives bit-identical results to launching every kernel directly (also with
    the complex64 basis storage)."""
    L, site, t, U = 6, 3, 1.0, 4.0
    print(f"krylov graph replay prec={prec} basis storage {storage}", flush=True)
    bonds, sites, model, (Lenv, Ld), (Renv, Rd) = _physical_envs(ctx, L, site, 2, 7, t, U, 24)
    left, right = bonds[site - 1], bonds[site + 1]
    bl, br = T.Bond(left), T.Bond(right)
    xk, xo, xt, xd = T.center_layout(bl, br, 2)
    xs = keyed(xk, random_blocks(xk, xd, 56))
    nrm = np.sqrt(sum(np.sum(np.abs(a) ** 2) for a in xs))
    x0 = pack([a / nrm for a in xs], xo, xt)
    out = {}
    ctx.set_precision(prec)
    ctx.set_krylov_storage(storage)
    try:
        for graphs in (False, True, False, True):
            ctx.set_graphs(graphs)
            x_d = dev(x0)
            rc, info = ctx.krylov_expm(model, site, 2, bl, br, T.Blocks(Ld[0], Ld[1], Lenv.data_ptr(), Ld[2]),
                                       T.Blocks(Rd[0], Rd[1], Renv.data_ptr(), Rd[2]),
                                       T.Blocks(xk, xo, x_d.data_ptr(), xt), -0.3j, tol=1e-13, maxdim=40)
            assert info["converged"], info
            print(f"  graphs={graphs} iters={info['iters']} replayed={info['graph_iters']}", flush=True)
            if graphs:   # FP64 captures once the tiling autotuner has settled, FP32 from the second iteration
                assert info["graph_iters"] > 0
                if prec == T.FP32:
                    assert info["graph_iters"] == info["iters"] - 1
            else:
                assert info["graph_iters"] == 0
            res = (host(x_d), info["alpha"], info["beta"])
            if graphs in out:
                assert np.array_equal(out[graphs][0], res[0])
            out[graphs] = res
    finally:
        ctx.set_graphs(True)
        ctx.set_precision(T.FP64)
        ctx.set_krylov_storage(T.FP64)
    assert np.array_equal(out[False][0], out[True][0])
    assert out[False][1] == out[True][1] and out[False][2] == out[True][2]


# --------------------------------------------------------------------------
# Error paths forced from the host (every kernel still runs to completion)
# --------------------------------------------------------------------------
def _apply_case(ctx, seed, poison=None):
    """Two-site apply on random blocks; poison = (index, value) planted in x."""
    left, right, bl, br, X, Lx, Rx = _heff_case(3, 2, seed)
    xk, xo, xt, xd, xs = X
    lk, lo, lt, ld, Ls = Lx
    rk, ro, rt, rd, Rs = Rx
    xb = pack(xs, xo, xt)
    if poison is not None:
        xb[poison[0]] = poison[1]
    x_d, L_d, R_d = dev(xb), dev(pack(Ls, lo, lt)), dev(pack(Rs, ro, rt))
    y_d = torch.zeros_like(x_d)
    ctx.heff_apply(T.Model(8), 3, 2, bl, br, T.Blocks(lk, lo, L_d.data_ptr(), lt),
                   T.Blocks(rk, ro, R_d.data_ptr(), rt), T.Blocks(xk, xo, x_d.data_ptr(), xt),
                   T.Blocks(xk, xo, y_d.data_ptr(), xt))
    return (x_d, L_d, R_d, y_d), (bl, br, xk, xo, xt, lk, lo, lt, rk, ro, rt)


@pytest.mark.parametrize("value", [float("nan"), float("inf")])
def test_nonfinite_input_surfaces_at_the_next_synchronisation(ctx, value):
    """A NaN or Inf in the input of an apply makes the next synchronising call
    return NONFINITE (-7), once: the flag is cleared and later clean work
    synchronises normally."""
    print(f"non-finite apply input {value}", flush=True)
    keep, _ = _apply_case(ctx, 410, poison=(17, value))
    with pytest.raises(T.TdvpError) as e:
        ctx.synchronize()
    assert e.value.code == -7
    keep, _ = _apply_case(ctx, 411)
    ctx.synchronize()
    assert np.isfinite(host(keep[3])).all()


def test_nonfinite_environment_in_env_update(ctx):
    print("non-finite environment in env update", flush=True)
    site = 4
    bin_, bout = _bond((site - 1) % 2, 300), _bond(site % 2, 301)
    bi, bo = T.Bond(bin_), T.Bond(bout)
    tk, to, tt, td = T.center_layout(bi, bo, 1)
    ek, eo, et, ed = T.env_layout(bi)
    ok, oo, ot, od = T.env_layout(bo)
    eb = pack(keyed(ek, random_blocks(ek, ed, 303)), eo, et)
    eb[et // 2] = complex(float("inf"), 0.0)
    t_d, e_d = dev(pack(keyed(tk, random_blocks(tk, td, 302)), to, tt)), dev(eb)
    o_d = torch.zeros(max(ot, 1), dtype=torch.complex128, device="cuda")
    ctx.env_update(T.Model(8), site, 1, bi, bo, T.Blocks(ek, eo, e_d.data_ptr(), et),
                   T.Blocks(tk, to, t_d.data_ptr(), tt), T.Blocks(ok, oo, o_d.data_ptr(), ot))
    with pytest.raises(T.TdvpError) as e:
        ctx.synchronize()
    assert e.value.code == -7
    ctx.synchronize()


def test_krylov_nonfinite_start_vector(ctx):
    print("krylov with a NaN in the start vector", flush=True)
    keep, (bl, br, xk, xo, xt, lk, lo, lt, rk, ro, rt) = _apply_case(ctx, 412)
    ctx.synchronize()
    x_d, L_d, R_d, _ = keep
    x_d[5] = complex(float("nan"), 0.0)
    rc, _ = ctx.krylov_expm(T.Model(8), 3, 2, bl, br, T.Blocks(lk, lo, L_d.data_ptr(), lt),
                            T.Blocks(rk, ro, R_d.data_ptr(), rt), T.Blocks(xk, xo, x_d.data_ptr(), xt),
                            -0.025j, tol=1e-12, maxdim=10, check=False)
    assert rc == -7
    ctx.synchronize()


def test_krylov_noconv_leaves_the_best_iterate(ctx):
    """maxdim = 2 with tol 1e-12 cannot converge: NOCONV (-6), and x holds the
    two-dimensional Krylov approximation, as the oracle's Lanczos gives it."""
    L, site, t, U = 6, 3, 1.0, 4.0
    print("krylov NOCONV at maxdim 2", flush=True)
    bonds, sites, model, (Lenv, Ld), (Renv, Rd) = _physical_envs(ctx, L, site, 2, 7, t, U, 24)
    left, right = bonds[site - 1], bonds[site + 1]
    bl, br = T.Bond(left), T.Bond(right)
    xk, xo, xt, xd = T.center_layout(bl, br, 2)
    xs = keyed(xk, random_blocks(xk, xd, 57))
    nrm = np.sqrt(sum(np.sum(np.abs(a) ** 2) for a in xs))
    xs = [a / nrm for a in xs]
    x_d = dev(pack(xs, xo, xt))
    rc, info = ctx.krylov_expm(model, site, 2, bl, br, T.Blocks(Ld[0], Ld[1], Lenv.data_ptr(), Ld[2]),
                               T.Blocks(Rd[0], Rd[1], Renv.data_ptr(), Rd[2]),
                               T.Blocks(xk, xo, x_d.data_ptr(), xt), -0.3j, tol=1e-12, maxdim=2, check=False)
    assert rc == -6 and info["iters"] == 2 and not info["converged"]
    ys = unpack(host(x_d), xo, xd)
    full = [R.expand_site("A" if k < site else ("C" if k == site else "B"), sites[k - 1], bonds[k - 1],
                          bonds[k], k) for k in range(1, L + 1)]
    Lf = D.empty_env()
    for k in range(1, site):
        Lf = D.left_env_update(Lf, full[k - 1], k, t, U)
    Rf = D.empty_env()
    for k in range(L, site + 1, -1):
        Rf = D.right_env_update(Rf, full[k - 1], k, t, U)
    v = R.expand_theta(theta_dict(xk, xs), left, right, site)
    ref, rinfo = D.lanczos_expm(lambda z: D.heff2(Lf, Rf, z, site, t, U), v, -0.3j, tol=1e-12, maxdim=2)
    assert rinfo["iters"] == 2 and not rinfo["converged"]
    got = R.expand_theta(theta_dict(xk, ys), left, right, site)
    assert np.abs(got - ref).max() < 1e-12


def test_nomem_from_a_capped_allocator():
    """A device allocator that refuses large requests makes the call that
    needs the memory return NOMEM (-4); the context stays usable."""
    import ctypes
    print("capped allocator: NOMEM", flush=True)
    stream = torch_stream_handle()
    cap = 4 << 20
    refused = []

    def alloc(n, user):
        if n > cap:
            refused.append(n)
            return None
        return torch.cuda.caching_allocator_alloc(int(n), 0, int(stream))

    def free(p, user):
        torch.cuda.caching_allocator_delete(int(p))

    cbs = (T._ALLOC_FN(alloc), T._FREE_FN(free))
    c = T.Context(0, stream=stream, allocator=cbs)
    try:
        keep, (bl, br, xk, xo, xt, lk, lo, lt, rk, ro, rt) = _apply_case(c, 413)
        c.synchronize()
        x_d, L_d, R_d, _ = keep
        assert 42 * 16 * xt > cap
        rc, _ = c.krylov_expm(T.Model(8), 3, 2, bl, br, T.Blocks(lk, lo, L_d.data_ptr(), lt),
                              T.Blocks(rk, ro, R_d.data_ptr(), rt), T.Blocks(xk, xo, x_d.data_ptr(), xt),
                              -0.025j, tol=1e-12, maxdim=40, check=False)
        assert rc == -4 and refused
        keep, _ = _apply_case(c, 414)    # small requests still succeed
        c.synchronize()
        assert np.isfinite(host(keep[3])).all()
    finally:
        c.close()


def test_heff_tilings_and_persistent_launch_are_bit_identical(monkeypatch):
    """Every FP64 candidate of the tiling autotuner -- mixed, all-32x32 and
    all-64x64 tiles, the all-64x64 tiles in a persistent launch that takes
    them from a device counter, and the all-32x32 tiles as wave tiles (one
    per wave, operands loaded straight into registers) -- gives the same bits
    (each element keeps its summation order whichever workgroup computes it)."""
    print("FP64 tilings and the persistent launch", flush=True)
    left, right, bl, br, X, Lx, Rx = _heff_case(4, 2, 500)
    xk, xo, xt, xd, xs = X
    lk, lo, lt, ld, Ls = Lx
    rk, ro, rt, rd, Rs = Rx
    x_d, L_d, R_d = dev(pack(xs, xo, xt)), dev(pack(Ls, lo, lt)), dev(pack(Rs, ro, rt))
    c = T.Context(0, stream=torch_stream_handle())
    outs = {}
    try:
        for mode in (2, 3, 0, 1, 4, 3, 4):
            monkeypatch.setenv("TDVP_FORCE_TILING", str(mode))
            y_d = torch.full_like(x_d, float("nan"))
            c.heff_apply(T.Model(8), 4, 2, bl, br, T.Blocks(lk, lo, L_d.data_ptr(), lt),
                         T.Blocks(rk, ro, R_d.data_ptr(), rt), T.Blocks(xk, xo, x_d.data_ptr(), xt),
                         T.Blocks(xk, xo, y_d.data_ptr(), xt))
            c.synchronize()
            y = host(y_d)
            assert np.isfinite(y).all()
            if mode in outs:
                assert np.array_equal(outs[mode], y)
            outs[mode] = y
    finally:
        monkeypatch.delenv("TDVP_FORCE_TILING", raising=False)
        c.close()
    for mode in (3, 0, 1, 4):
        assert np.array_equal(outs[2], outs[mode]), mode


def test_fp32_tilings_are_bit_identical(monkeypatch):
    """FP32 block products (energy shift included) on every tiling the FP32
    launches can take -- mixed, all-32x32 and all-64x64 LDS-staged tiles and
    the wave tiles -- give the same bits: the products of each element come
    in the same order, from the same FP32 values."""
    print("FP32 tilings", flush=True)
    left, right, bl, br, X, Lx, Rx = _heff_case(4, 2, 501)
    xk, xo, xt, xd, xs = X
    lk, lo, lt, ld, Ls = Lx
    rk, ro, rt, rd, Rs = Rx
    x_d, L_d, R_d = dev(pack(xs, xo, xt)), dev(pack(Ls, lo, lt)), dev(pack(Rs, ro, rt))
    c = T.Context(0, stream=torch_stream_handle(), precision=T.FP32)
    outs = {}
    try:
        for mode in (2, 4, 0, 1):
            monkeypatch.setenv("TDVP_FORCE_TILING", str(mode))
            y_d = torch.full_like(x_d, float("nan"))
            c.heff_apply(T.Model(8), 4, 2, bl, br, T.Blocks(lk, lo, L_d.data_ptr(), lt),
                         T.Blocks(rk, ro, R_d.data_ptr(), rt), T.Blocks(xk, xo, x_d.data_ptr(), xt),
                         T.Blocks(xk, xo, y_d.data_ptr(), xt))
            c.synchronize()
            outs[mode] = host(y_d)
            assert np.isfinite(outs[mode]).all()
    finally:
        monkeypatch.delenv("TDVP_FORCE_TILING", raising=False)
        c.close()
    diffs = {m: float(np.abs(outs[m] - outs[2]).max()) for m in (4, 0, 1)}
    print("  max |difference| to the all-64x64 tiles:", diffs, flush=True)
    for mode in (4, 0, 1):
        assert np.array_equal(outs[2], outs[mode]), mode
