"""GPU parity of the abelian U(1) x U(1) variant (the paper's comparison
symmetry) through the C ABI: effective-Hamiltonian applies (one and two
sites, FP64 / FP32 / split-BF16 block products), environment updates (both
directions) and the Krylov exponential, against the oracle's dense
definitions on the full tensors.

Sizes: bonds of ~10-30 sectors with one degeneracy of ~70 (blocks spanning
several 64x64 tiles with ragged tails) while the dense expansion still fits
in seconds."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2606_04771_amd as T
from oracle import abelian as A
from oracle import dense as D
import synth
from tests._harness import torch_stream_handle, keyed, pack, random_blocks, theta_dict, env_dict, unpack

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 4e-6


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    c = T.Context(0, stream=torch_stream_handle())
    yield c
    c.close()


def dev(buf):
    return torch.from_numpy(buf).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("nsites,prec", [(2, T.FP64), (2, T.FP32), (2, T.BF16X3), (1, T.FP64), (1, T.FP32)])
def test_u1_heff_apply_against_oracle(ctx, nsites, prec):
    site, t, U = 4, 1.0, 4.0
    print(f"u1 heff nsites={nsites} prec={prec}", flush=True)
    left = synth.u1_profile(60, 70, site - 1, window=3, big=72)
    right = synth.u1_profile(60, 71, site + nsites - 1, window=3, big=66)
    bl, br = T.Bond(left), T.Bond(right)
    xk, xo, xt, xd = T.center_layout(bl, br, nsites, abelian=True)
    lk, lo, lt, ld = T.env_layout(bl, abelian=True)
    rk, ro, rt, rd = T.env_layout(br, abelian=True)
    xs = keyed(xk, random_blocks(xk, xd, 72))
    Ls = keyed(lk, random_blocks(lk, ld, 73))
    Rs = keyed(rk, random_blocks(rk, rd, 74))
    x_d, L_d, R_d = dev(pack(xs, xo, xt)), dev(pack(Ls, lo, lt)), dev(pack(Rs, ro, rt))
    y_d = torch.full_like(x_d, float("nan"))
    ctx.set_precision(prec)
    try:
        ctx.heff_apply(T.Model(8, t, U), site, nsites, bl, br, T.Blocks(lk, lo, L_d.data_ptr(), lt),
                       T.Blocks(rk, ro, R_d.data_ptr(), rt), T.Blocks(xk, xo, x_d.data_ptr(), xt),
                       T.Blocks(xk, xo, y_d.data_ptr(), xt), abelian=True)
        ctx.synchronize()
        ys = unpack(host(y_d), xo, xd)
    finally:
        ctx.set_precision(T.FP64)
    Lf = A.expand_env(env_dict(lk, Ls), left)
    Rf = A.expand_env(env_dict(rk, Rs), right)
    if nsites == 2:
        ref = D.heff2(Lf, Rf, A.expand_theta(theta_dict(xk, xs), left, right), site, t, U)
        got = A.expand_theta(theta_dict(xk, ys), left, right)
    else:
        ref = D.heff1(Lf, Rf, A.expand_site(theta_dict(xk, xs), left, right), site, t, U)
        got = A.expand_site(theta_dict(xk, ys), left, right)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  {len(xk)} blocks, max error relative to the largest entry {err:.2e}", flush=True)
    assert err < (FP64_TOL if prec == T.FP64 else FP32_TOL)


@pytest.mark.parametrize("direction,prec", [(1, T.FP64), (-1, T.FP64), (1, T.FP32), (-1, T.BF16X3)])
def test_u1_env_update_against_oracle(ctx, direction, prec):
    site, t, U = 4, 1.0, 4.0
    print(f"u1 env update direction={direction} prec={prec}", flush=True)
    b_left = synth.u1_profile(50, 80, site - 1, window=3, big=70)
    b_right = synth.u1_profile(50, 81, site, window=3, big=68)
    if direction > 0:
        bin_, bout = b_left, b_right
        tk, to, tt, td = T.center_layout(T.Bond(bin_), T.Bond(bout), 1, abelian=True)
    else:
        bin_, bout = b_right, b_left
        tk, to, tt, td = T.center_layout(T.Bond(bout), T.Bond(bin_), 1, abelian=True)
    bi, bo = T.Bond(bin_), T.Bond(bout)
    ek, eo, et, ed = T.env_layout(bi, abelian=True)
    ok, oo, ot, od = T.env_layout(bo, abelian=True)
    ts = keyed(tk, random_blocks(tk, td, 82))
    Es = keyed(ek, random_blocks(ek, ed, 83))
    t_d, e_d = dev(pack(ts, to, tt)), dev(pack(Es, eo, et))
    o_d = torch.full((max(ot, 1),), float("nan"), dtype=torch.complex128, device="cuda")
    ctx.set_precision(prec)
    try:
        ctx.env_update(T.Model(8, t, U), site, direction, bi, bo, T.Blocks(ek, eo, e_d.data_ptr(), et),
                       T.Blocks(tk, to, t_d.data_ptr(), tt), T.Blocks(ok, oo, o_d.data_ptr(), ot), abelian=True)
        ctx.synchronize()
        outs = unpack(host(o_d), oo, od)
    finally:
        ctx.set_precision(T.FP64)
    Ef = A.expand_env(env_dict(ek, Es), bin_)
    if direction > 0:
        ref = D.left_env_update(Ef, A.expand_site(theta_dict(tk, ts), bin_, bout), site, t, U)
    else:
        ref = D.right_env_update(Ef, A.expand_site(theta_dict(tk, ts), bout, bin_), site, t, U)
    got = A.expand_env(env_dict(ok, outs), bout)
    scale = max(np.abs(ref[w]).max() for w in range(3))
    err = max(np.abs(got[w] - ref[w]).max() for w in range(3)) / scale
    print(f"  max error relative to the largest entry {err:.2e}", flush=True)
    assert err < (FP64_TOL if prec == T.FP64 else FP32_TOL)


@pytest.mark.parametrize("nsites,tau", [(2, -0.1j), (1, 0.05j)])
def test_u1_krylov_against_oracle(ctx, nsites, tau):
    """Environments of a seeded random U(1) x U(1) chain (L = 6, sites 1..site-1
    and site+nsites..L contracted by the oracle's dense updates, so the
    effective Hamiltonian is Hermitian), cut into sector blocks; the library's
    Krylov exponential against the oracle's on the full tensors."""
    L, site, t, U = 6, 3, 1.0, 4.0
    print(f"u1 krylov nsites={nsites} tau={tau}", flush=True)
    bonds = [[(0, 0, 1)]] + [synth.u1_profile(14, 90 + k, k, window=2) for k in range(1, L)] + [[(0, L, 1)]]
    Tb = [T.Bond(b) for b in bonds]
    sites = []
    for k in range(1, L + 1):
        tk, to, tt, td = T.center_layout(Tb[k - 1], Tb[k], 1, abelian=True)
        blocks = random_blocks(tk, td, 95, k)
        sites.append(A.expand_site({tuple(int(v) for v in kk): b for kk, b in blocks.items()}, bonds[k - 1], bonds[k]))
    Lf = D.empty_env()
    for k in range(1, site):
        Lf = D.left_env_update(Lf, sites[k - 1], k, t, U)
    Rf = D.empty_env()
    for k in range(L, site + nsites - 1, -1):
        Rf = D.right_env_update(Rf, sites[k - 1], k, t, U)
    left, right = bonds[site - 1], bonds[site + nsites - 1]
    bl, br = Tb[site - 1], Tb[site + nsites - 1]
    lk, lo, lt, ld = T.env_layout(bl, abelian=True)
    rk, ro, rt, rd = T.env_layout(br, abelian=True)
    Ls = A.restrict_env(Lf, left, [tuple(int(v) for v in k) for k in lk])
    Rs = A.restrict_env(Rf, right, [tuple(int(v) for v in k) for k in rk])
    xk, xo, xt, xd = T.center_layout(bl, br, nsites, abelian=True)
    xs = keyed(xk, random_blocks(xk, xd, 96))
    nrm = np.sqrt(sum(np.sum(np.abs(a) ** 2) for a in xs))
    xs = [a / nrm for a in xs]
    L_d = dev(pack([Ls[tuple(int(v) for v in k)] for k in lk], lo, lt))
    R_d = dev(pack([Rs[tuple(int(v) for v in k)] for k in rk], ro, rt))
    x_d = dev(pack(xs, xo, xt))
    rc, info = ctx.krylov_expm(T.Model(L, t, U), site, nsites, bl, br, T.Blocks(lk, lo, L_d.data_ptr(), lt),
                               T.Blocks(rk, ro, R_d.data_ptr(), rt), T.Blocks(xk, xo, x_d.data_ptr(), xt), tau,
                               tol=1e-13, maxdim=40, abelian=True)
    assert info["converged"], info
    ys = unpack(host(x_d), xo, xd)
    if nsites == 2:
        v = A.expand_theta(theta_dict(xk, xs), left, right)
        ref, _ = D.lanczos_expm(lambda z: D.heff2(Lf, Rf, z, site, t, U), v, tau, tol=1e-15, maxdim=60)
        got = A.expand_theta(theta_dict(xk, ys), left, right)
    else:
        v = A.expand_site(theta_dict(xk, xs), left, right)
        ref, _ = D.lanczos_expm(lambda z: D.heff1(Lf, Rf, z, site, t, U), v, tau, tol=1e-15, maxdim=60)
        got = A.expand_site(theta_dict(xk, ys), left, right)
    err = np.abs(got - ref).max()
    print(f"  iters={info['iters']} err={err:.2e}", flush=True)
    assert err < 1e-10
    assert abs(np.linalg.norm(got) - 1.0) < 1e-12


# ---- U(1) x U(1) chains: sweeps, observables and overlaps ---------------------

def u1_state(mps, L):
    """Expand a library U(1) x U(1) MPS (centre on site 1) with the oracle's
    abelian conventions and contract it to a state vector."""
    bonds = [mps.bond(k) for k in range(L + 1)]
    full = []
    for k in range(1, L + 1):
        keys, offs, data = mps.site(k)
        dims = [(bonds[k - 1][kk[0]][2], bonds[k][kk[2]][2]) for kk in keys]
        full.append(A.expand_site(theta_dict(keys, unpack(data, offs, dims)), bonds[k - 1], bonds[k]))
    return D.mps_state(full)


def u1_library_mps(ctx, model, bonds, sites):
    Tb = [T.Bond(b) for b in bonds]
    bufs, descs = [], []
    for k in range(1, len(sites) + 1):
        tk, to, tt, _ = T.center_layout(Tb[k - 1], Tb[k], 1, abelian=True)
        d = dev(pack([sites[k - 1][tuple(int(v) for v in kk)] for kk in tk], to, tt))
        bufs.append(d)
        descs.append(T.Blocks(tk, to, d.data_ptr(), tt))
    mps = T.MPS.from_blocks(ctx, model, Tb, descs, abelian=True)
    torch.cuda.synchronize()
    return mps


def u1_oracle_mps(bonds, sites):
    return [A.expand_site(sites[k - 1], bonds[k - 1], bonds[k]) for k in range(1, len(sites) + 1)]


def test_u1_neel_mps_is_the_neel_state(ctx):
    from oracle import fermions as F
    L = 6
    for complete in (False, True):
        mps = T.MPS.neel(ctx, T.Model(L, 1.0, 4.0), complete=complete, abelian=True)
        assert mps.bond(L) == [(0, L, 1)]
        psi = u1_state(mps, L)
        assert abs(abs(np.vdot(F.neel_state(L), psi)) - 1) < 1e-14
        sz, docc, n2 = mps.measure()
        assert np.abs(sz - 0.5 * (-1.0) ** np.arange(L)).max() < 1e-14
        assert np.abs(docc).max() < 1e-14 and abs(n2 - 1) < 1e-14
        mps.close()


@pytest.mark.parametrize("one_site", [False, True])
def test_u1_complete_basis_sweeps_follow_exact_evolution_L8(ctx, one_site):
    """L = 8 Neel quench (U/J = 4, dt = 0.05) with every bond at its full
    U(1) x U(1) dimension, where two-site and one-site TDVP are exact:
    against the 4^8 state-vector evolution, with the library's own
    observables (S^z, double occupancy, norm)."""
    from oracle import fermions as F
    L, t, U, dt, nsteps = 8, 1.0, 4.0, 0.05, 20
    mps = T.MPS.neel(ctx, T.Model(L, t, U), complete=True, abelian=True)
    exact = F.evolve(F.hubbard(L, t, U), F.neel_state(L), np.arange(nsteps + 1) * dt)
    worst = 0.0
    for n in range(1, nsteps + 1):
        if one_site:
            info = mps.sweep1(dt, krylov_tol=1e-14, krylov_maxdim=50)
        else:
            info = mps.sweep(dt, keep_all=True, krylov_tol=1e-14, krylov_maxdim=50)
        assert info["nonconverged"] == 0
        if n % 5 == 0 or n == 1:
            psi = u1_state(mps, L)
            nu0, nd0, dd0 = F.local_expectations(exact[n], L)
            nu, nd, dd = F.local_expectations(psi, L)
            sz, docc, n2 = mps.measure()
            err = max(abs(1 - abs(np.vdot(exact[n], psi))), np.abs(nu - nu0).max(), np.abs(dd - dd0).max(),
                      np.abs(sz - 0.5 * (nu0 - nd0)).max(), np.abs(docc - dd0).max(), abs(n2 - 1))
            print(f"t={n * dt:.2f} err {err:.2e} chi {info['max_chi']} krylov {info['krylov_iters']}", flush=True)
            worst = max(worst, err)
    mps.close()
    assert worst < 1e-10


@pytest.mark.parametrize("chi_cap,eps", [(24, 1e-8), (40, 1e-3)])
def test_u1_truncated_sweeps_match_oracle(ctx, chi_cap, eps):
    """Truncated two-site TDVP from a seeded random U(1) x U(1) MPS (L = 8):
    the library's per-sector split keeps single singular values by the same
    rule as the oracle's plain truncated SVD of the dense two-site matrix, so
    the states, the discarded weights and the observables agree."""
    from oracle import fermions as F
    L, t, U, dt = 8, 1.0, 4.0, 0.05
    bonds, sites = synth.u1_random_mps(L, 48, 17)
    mps = u1_library_mps(ctx, T.Model(L, t, U), bonds, sites)
    ref = u1_oracle_mps(bonds, sites)
    assert abs(np.linalg.norm(D.mps_state(ref)) - 1) < 1e-12
    assert abs(np.vdot(D.mps_state(ref), u1_state(mps, L)) - 1) < 1e-12
    for n in range(3):
        info = mps.sweep(dt, eps_tol=eps, chi_cap=chi_cap, keep_all=False, krylov_tol=1e-14, krylov_maxdim=50)
        ref, disc = D.tdvp2_sweep(ref, dt, t, U, tol=1e-14, maxdim=50, keep_all=False, eps_tol=eps, chi_cap=chi_cap)
        psi, phi = u1_state(mps, L), D.mps_state(ref)
        ov = abs(np.vdot(phi, psi))
        nu, nd, dd = F.local_expectations(psi, L)
        mu, md, de = F.local_expectations(phi, L)
        sz, docc, n2 = mps.measure()
        print(f"sweep {n + 1}: 1-|ov| {1 - ov:.2e} chi {info['max_chi']} max disc {info['max_discarded']:.2e} "
              f"(oracle {max(disc):.2e})", flush=True)
        assert info["max_chi"] <= chi_cap
        assert abs(info["max_discarded"] - max(disc)) < 1e-10
        assert 1 - ov < 1e-10
        assert max(np.abs(nu - mu).max(), np.abs(nd - md).max(), np.abs(dd - de).max()) < 1e-10
        assert np.abs(sz - 0.5 * (nu - nd)).max() < 1e-12 and np.abs(docc - dd).max() < 1e-12
    mps.close()


def test_u1_one_site_sweeps_and_overlap_match_oracle(ctx):
    """One-site TDVP at fixed bond dimensions from a seeded random U(1) x U(1)
    MPS against the oracle's dense one-site sweep, and the overlap of two
    such chains against the vdot of their expanded state vectors."""
    L, t, U, dt = 8, 1.0, 4.0, 0.05
    bonds, sites = synth.u1_random_mps(L, 48, 23)
    b2, s2 = synth.u1_random_mps(L, 24, 29)
    model = T.Model(L, t, U)
    mps, other = u1_library_mps(ctx, model, bonds, sites), u1_library_mps(ctx, model, b2, s2)
    ref = u1_oracle_mps(bonds, sites)
    psi2 = D.mps_state(u1_oracle_mps(b2, s2))
    assert abs(other.overlap(mps) - np.vdot(psi2, D.mps_state(ref))) < 1e-13
    for n in range(3):
        info = mps.sweep1(dt, krylov_tol=1e-14, krylov_maxdim=50)
        ref = D.tdvp1_sweep(ref, dt, t, U, tol=1e-14, maxdim=50)
        psi, phi = u1_state(mps, L), D.mps_state(ref)
        ov = abs(np.vdot(phi, psi))
        print(f"sweep {n + 1}: 1-|ov| {1 - ov:.2e} krylov {info['krylov_iters']}", flush=True)
        assert 1 - ov < 1e-10
        assert mps.bond(4) == [tuple(b) for b in bonds[4]]
        assert abs(other.overlap(mps) - np.vdot(psi2, psi)) < 1e-12
    mps.close()
    other.close()


def test_u1_host_staged_sweeps_and_adaptive_step():
    """U(1) x U(1) chains with the memory plan (inactive tensors in host
    memory, FP64 Krylov storage) give bit-identical sweeps, and
    the library's adaptive step switches to one-site sweeps once the largest
    bond reaches the given fraction of the cap, on a seeded L = 12 chain."""
    L, t, U, dt = 12, 1.0, 4.0, 0.05
    bonds, sites = synth.u1_random_mps(L, 40, 31)
    model = T.Model(L, t, U)
    c1 = T.Context(0, stream=torch_stream_handle())
    c2 = T.Context(0, stream=torch_stream_handle())
    c2.set_host_staging(True)
    try:
        m1, m2 = u1_library_mps(c1, model, bonds, sites), u1_library_mps(c2, model, bonds, sites)
        for n in range(2):
            i1 = m1.sweep(dt, eps_tol=1e-8, chi_cap=48, krylov_tol=1e-12, krylov_maxdim=40)
            i2 = m2.sweep(dt, eps_tol=1e-8, chi_cap=48, krylov_tol=1e-12, krylov_maxdim=40)
            assert i1["max_chi"] == i2["max_chi"] and i1["krylov_iters"] == i2["krylov_iters"]
        for k in range(1, L + 1):
            k1, o1, d1 = m1.site(k)
            k2, o2, d2 = m2.site(k)
            assert np.array_equal(k1, k2) and np.array_equal(d1, d2)
        sz1, dd1, _ = m1.measure()
        sz2, dd2, _ = m2.measure()
        assert np.array_equal(sz1, sz2) and np.array_equal(dd1, dd2)
        # adaptive step: cap 24, switch at 75 % of it
        mode, modes = 0, []
        for n in range(4):
            info, mode = m1.step(dt, mode, eps_tol=1e-8, chi_cap=24, krylov_tol=1e-12, krylov_maxdim=40, switch=0.75)
            modes.append(mode)
            assert info["max_chi"] <= 24
        print("modes", modes, flush=True)
        assert modes[-1] == 1
        m1.close()
        m2.close()
    finally:
        c1.close()
        c2.close()
