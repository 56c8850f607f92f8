"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, an independent library, invariants, brute force, or a value printed
in the paper.  A plausible slip anywhere in the oracle (a dropped term, a
wrong sign or index, a transposed operand) breaks at least one of them.
"""
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import cg as CG
from oracle import dense as D
from oracle import fermions as F
from oracle import reduced as R
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Clebsch-Gordan coefficients
# --------------------------------------------------------------------------
def test_cg_matches_sympy():
    from sympy import S
    from sympy.physics.wigner import clebsch_gordan
    worst = 0.0
    for tj1 in range(0, 6):
        for tj2 in range(0, 5):
            for tJ in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2):
                for tm1 in range(-tj1, tj1 + 1, 2):
                    for tm2 in range(-tj2, tj2 + 1, 2):
                        tM = tm1 + tm2
                        if abs(tM) > tJ:
                            continue
                        ref = float(clebsch_gordan(S(tj1) / 2, S(tj2) / 2, S(tJ) / 2,
                                                   S(tm1) / 2, S(tm2) / 2, S(tM) / 2))
                        worst = max(worst, abs(CG.cg2(tj1, tm1, tj2, tm2, tJ, tM) - ref))
    assert worst < 1e-15


def test_cg_closed_forms_and_orthonormality():
    # coupling to a singlet: <j m; j -m | 0 0> = (-1)^(j-m) / sqrt(2j+1)
    for tj in range(0, 9):
        for tm in range(-tj, tj + 1, 2):
            ref = (-1) ** ((tj - tm) // 2) / np.sqrt(tj + 1)
            assert abs(CG.cg2(tj, tm, tj, -tm, 0, 0) - ref) < 1e-15
    # stretched state <j1 j1; j2 j2 | j1+j2 j1+j2> = 1
    for tj1 in range(0, 7):
        for tj2 in range(0, 7):
            assert abs(CG.cg2(tj1, tj1, tj2, tj2, tj1 + tj2, tj1 + tj2) - 1.0) < 1e-15
    # unitarity of the coupling transformation
    for tj1 in range(0, 6):
        for tj2 in range(0, 4):
            rows = []
            for tJ in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2):
                rows.append(CG.cg_tensor(tj1, tj2, tJ).reshape(-1, tJ + 1))
            Umat = np.concatenate(rows, axis=1)
            assert np.allclose(Umat.T @ Umat, np.eye(Umat.shape[1]), atol=1e-14)


# --------------------------------------------------------------------------
# Fermions, Hamiltonian, pseudospin
# --------------------------------------------------------------------------
def test_jordan_wigner_anticommutation():
    L = 3
    c = [F.annihilator(i, s, L) for i in range(1, L + 1) for s in (0, 1)]
    eye = np.eye(4 ** L)
    for p in range(len(c)):
        for q in range(len(c)):
            ac = (c[p] @ c[q].T + c[q].T @ c[p]).toarray()
            assert np.allclose(ac, eye * (p == q))
            aa = (c[p] @ c[q] + c[q] @ c[p]).toarray()
            assert np.allclose(aa, 0.0)


def test_pseudospin_algebra_and_symmetry_of_h():
    """Supplementary S2.1: [T+,T-] = 2Tz, [Tz,T+-] = +-T+-; the symmetric
    interaction commutes with T+, Eq. (1)'s n_up n_dn gives [H,T+] = U T+."""
    L = 4
    U = 3.0
    Tp, Tm, Tz = F.pseudospin(L)
    assert abs(Tp @ Tm - Tm @ Tp - 2 * Tz).max() < 1e-12
    assert abs(Tz @ Tp - Tp @ Tz - Tp).max() < 1e-12
    assert abs(Tz @ Tm - Tm @ Tz + Tm).max() < 1e-12
    Hs = F.hubbard(L, 1.0, U, symmetric=True)
    He = F.hubbard(L, 1.0, U, symmetric=False)
    assert abs(Hs @ Tp - Tp @ Hs).max() < 1e-12
    assert abs(He @ Tp - Tp @ He - U * Tp).max() < 1e-12


def test_neel_quantum_numbers():
    L = 6
    psi = F.neel_state(L)
    Tp, Tm, Tz = F.pseudospin(L)
    T2 = Tp @ Tm + Tz @ Tz - Tz
    assert abs(np.vdot(psi, T2 @ psi)) < 1e-14
    nu, nd, _ = F.local_expectations(psi, L)
    assert np.allclose(nu, [1, 0, 1, 0, 1, 0]) and np.allclose(nd, 1 - nu)
    He = F.hubbard(L, 1.0, 4.0)
    Hs = F.hubbard(L, 1.0, 4.0, symmetric=True)
    assert abs(np.vdot(psi, He @ psi)) < 1e-14                      # E_Eq1(Neel) = 0
    assert abs(np.vdot(psi, Hs @ psi).real + 4.0 * L / 4) < 1e-12  # E_sym = -UL/4


def test_free_fermion_closed_form():
    """U = 0: each spin species evolves as free fermions on the open chain."""
    L = 6
    H = F.hubbard(L, 1.0, 0.0)
    psi0 = F.neel_state(L)
    times = np.linspace(0.0, 2.0, 5)
    traj = F.evolve(H, psi0, times)
    n0u = np.array([1.0 if i % 2 == 0 else 0.0 for i in range(L)])
    ref = F.free_fermion_density(L, 1.0, times, n0u)
    for k in range(len(times)):
        nu, nd, _ = F.local_expectations(traj[k], L)
        assert np.abs(nu - ref[k]).max() < 1e-12
        assert np.abs(nd - F.free_fermion_density(L, 1.0, [times[k]], 1 - n0u)[0]).max() < 1e-12


def test_short_time_expansion():
    """<n_i,up(t)> = n0 + (1 - 2 n0) z_i t^2 + O(t^4), independent of U."""
    L = 6
    for U in (0.0, 4.0):
        H = F.hubbard(L, 1.0, U)
        psi = F.evolve(H, F.neel_state(L), [0.0, 0.02])[1]
        nu, _, _ = F.local_expectations(psi, L)
        n0 = np.array([1.0 if i % 2 == 0 else 0.0 for i in range(L)])
        z = np.array([1] + [2] * (L - 2) + [1])
        ref = n0 + (1 - 2 * n0) * z * 0.02 ** 2
        assert np.abs(nu - ref).max() < 5e-6


def test_exact_invariants():
    L = 6
    U = 4.0
    H = F.hubbard(L, 1.0, U)
    traj = F.evolve(H, F.neel_state(L), [0.0, 0.5, 1.5])
    for psi in traj:
        nu, nd, dd = F.local_expectations(psi, L)
        assert np.abs(nu + nd - 1).max() < 1e-12                # <n_i> = 1
        assert np.abs(dd - (1 - nu - nd + dd)).max() < 1e-12    # doublon = holon
        assert np.abs(nu - nd[::-1]).max() < 1e-12              # reflection x spin flip
        assert abs(np.vdot(psi, H @ psi)) < 1e-12               # E_Eq1 conserved (= 0)
        assert abs(np.linalg.norm(psi) - 1) < 1e-12


def test_zero_hopping_is_static():
    L = 4
    H = F.hubbard(L, 0.0, 4.0)
    psi = F.evolve(H, F.neel_state(L), [0.0, 3.0])[1]
    nu, _, _ = F.local_expectations(psi, L)
    assert np.allclose(nu, [1, 0, 1, 0], atol=1e-14)


# --------------------------------------------------------------------------
# Reduced-tensor conventions
# --------------------------------------------------------------------------
def _expand_mps(bonds, sites, center):
    full = []
    for k in range(1, len(sites) + 1):
        kind = "A" if k < center else ("C" if k == center else "B")
        full.append(R.expand_site(kind, sites[k - 1], bonds[k - 1], bonds[k], k))
    return full


def test_reduced_expansion_isometries_and_singlet():
    L = 6
    bonds, sites = synth.random_mps(L, 24, seed=3, center=3)
    full = _expand_mps(bonds, sites, 3)
    for k in (1, 2):
        A = full[k - 1].reshape(-1, full[k - 1].shape[2])
        assert np.allclose(A.conj().T @ A, np.eye(A.shape[1]), atol=1e-13)
    for k in (4, 5, 6):
        B = full[k - 1].reshape(full[k - 1].shape[0], -1)
        assert np.allclose(B @ B.conj().T, np.eye(B.shape[0]), atol=1e-13)
    psi = D.mps_state(full)
    flat = np.sqrt(sum(np.sum(np.abs(v) ** 2) for v in sites[2].values()))
    assert abs(np.linalg.norm(psi) - flat) < 1e-13
    Tp, Tm, Tz = F.pseudospin(L)
    assert abs(np.vdot(psi, (Tp @ Tm + Tz @ Tz - Tz) @ psi)) < 1e-13
    nu, nd, _ = F.local_expectations(psi / np.linalg.norm(psi), L)
    assert abs(np.sum(nu - nd)) < 1e-13                          # S^z = 0


def _theta_keys_of(left, right):
    keys = []
    for ia, (qa, tja, da) in enumerate(left):
        for s1, (q1, t1) in enumerate(R.MULTIPLETS):
            for tjx in range(abs(tja - t1), tja + t1 + 1, 2):
                for s2, (q2, t2) in enumerate(R.MULTIPLETS):
                    for ib, (qb, tjb, db) in enumerate(right):
                        if qa + q1 + q2 == qb and abs(tjx - t2) <= tjb <= tjx + t2:
                            keys.append((ia, s1, tjx, s2, ib))
    return keys


def test_theta_expansion_is_a_singlet_with_the_flat_norm():
    """A state built from expanded left-canonical A's, an expanded random
    reduced two-site tensor and expanded right-canonical B's has S^z = 0 and
    T^2 = 0 exactly (the pseudospin singlet of section S2.1), and its norm is
    the flat norm of the reduced blocks.  A wrong fusion tree, a reversed
    magnetic order in one Clebsch-Gordan factor or a wrong normalisation
    breaks one of the three."""
    L, i = 6, 3
    bonds, sites = synth.random_mps(L, 30, seed=5, center=i)
    left, right = bonds[i - 1], bonds[i + 1]
    keys = _theta_keys_of(left, right)
    blocks = synth.block_data(keys, [(left[k[0]][2], right[k[4]][2]) for k in keys], seed=1)
    Th = R.expand_theta(blocks, left, right, i)
    full = [R.expand_site("A", sites[k - 1], bonds[k - 1], bonds[k], k) for k in range(1, i)]
    full.append(Th.reshape(Th.shape[0], 4, -1))       # sites i, i+1 as one [chi, 4, 4 chi] factor
    psi = full[0]
    for M in full[1:]:
        psi = np.tensordot(psi, M, axes=([psi.ndim - 1], [0]))
    psi = psi.reshape(-1, Th.shape[-1])
    tail = [R.expand_site("B", sites[k - 1], bonds[k - 1], bonds[k], k) for k in range(i + 2, L + 1)]
    rest = tail[0]
    for M in tail[1:]:
        rest = np.tensordot(rest, M, axes=([rest.ndim - 1], [0]))
    psi = (psi @ rest.reshape(rest.shape[0], -1)).reshape(-1)
    flat = np.sqrt(sum(np.sum(np.abs(b) ** 2) for b in blocks.values()))
    assert abs(np.linalg.norm(psi) - flat) < 1e-12 * flat
    assert abs(np.linalg.norm(Th) - flat) < 1e-12 * flat
    Tp, Tm, Tz = F.pseudospin(L)
    T2 = Tp @ Tm + Tz @ Tz - Tz
    assert np.linalg.norm(T2 @ psi) < 1e-12 * flat
    sz2 = sum(F.site_op(F.N_UP - F.N_DN, k, L) for k in range(1, L + 1))
    assert np.linalg.norm(sz2 @ psi) < 1e-12 * flat


def test_theta_tree_equals_merged_one_site_tensors():
    """The two-site tree ((a s1)->x) s2->b with its 1/sqrt(2j_b+1) is what the
    product of a one-site centre C(a, s1, x) and a right-canonical B(x, s2, b)
    expands to: Theta(a, s1, x, s2, b) = C(a, s1, x) B(x, s2, b) blockwise."""
    L, i = 6, 3
    bonds, sites = synth.random_mps(L, 30, seed=8, center=i)
    C = R.expand_site("C", sites[i - 1], bonds[i - 1], bonds[i], i)
    B = R.expand_site("B", sites[i], bonds[i], bonds[i + 1], i + 1)
    dense = np.tensordot(C, B, axes=([2], [0]))
    mid = bonds[i]
    red = {}
    for (ia, s1, ix), c in sites[i - 1].items():
        for (jx, s2, ib), b in sites[i].items():
            if jx == ix:
                key = (ia, s1, mid[ix][1], s2, ib)
                red[key] = red.get(key, 0) + c @ b
    Th = R.expand_theta(red, bonds[i - 1], bonds[i + 1], i)
    assert np.abs(Th - dense).max() < 1e-13


def test_row_operators_and_theta_labels():
    """The left part of every reduced block (a, s1, x, s2, b) carries the
    coupled label x: 2 S^z = q_x and T^2 = j_x (j_x + 1) on its rows.  The
    row operators built on the reduced bond (spin matrices of each sector)
    are the fermion operators projected on the block basis of expanded
    left-canonical tensors."""
    L, i = 6, 4
    bonds, sites = synth.random_mps(L, 26, seed=6, center=i)
    left, right = bonds[i - 1], bonds[i + 1]
    Sz2, T2 = R.row_quantum_ops(left, i)
    Afull = [R.expand_site("A", sites[k - 1], bonds[k - 1], bonds[k], k) for k in range(1, i)]
    Sz2_d, T2_d = D.left_row_ops(Afull + [None], i)
    assert np.abs(Sz2 - Sz2_d).max() < 1e-12 and np.abs(T2 - T2_d).max() < 1e-12
    keys = _theta_keys_of(left, right)
    for key in keys[::3]:
        blk = synth.complex_normal((left[key[0]][2], right[key[4]][2]), 2, *key)
        Th = R.expand_theta({key: blk}, left, right, i)
        M = Th.reshape(Th.shape[0] * 4, -1)
        qx = left[key[0]][0] + R.MULTIPLETS[key[1]][0]
        jx = key[2] / 2.0
        assert np.abs(Sz2 @ M - qx * M).max() < 1e-12 * np.abs(M).max()
        assert np.abs(T2 @ M - jx * (jx + 1) * M).max() < 1e-12 * np.abs(M).max()


def _project_env(E, bond):
    offs, _ = R.bond_offsets(bond)
    resid = 0.0
    for io, (qo, tjo, do) in enumerate(bond):
        for ii, (qi, tji, di) in enumerate(bond):
            for w, (qw, tjw) in enumerate(R.CHANNELS):
                sub = E[w][offs[io]:offs[io] + do * (tjo + 1), :, offs[ii]:offs[ii] + di * (tji + 1)]
                sub = sub.reshape(do, tjo + 1, tjw + 1, di, tji + 1)
                if qo != qi + qw or not (abs(tji - tjw) <= tjo <= tji + tjw):
                    resid = max(resid, np.abs(sub).max())
                    continue
                mt = np.transpose(CG.cg_tensor(tji, tjw, tjo), (2, 1, 0))
                blk = np.einsum("xakyb,akb->xy", sub, mt) / np.sum(mt ** 2)
                resid = max(resid, np.abs(np.einsum("xy,akb->xakyb", blk, mt) - sub).max())
    return resid


def test_environment_wigner_eckart_form():
    """Dense environments of an expanded symmetric MPS have exactly the
    documented reduced form E_red x C(j_in m; j_w kappa | j_out m')."""
    L = 6
    t, U = 1.0, 4.0
    bonds, sites = synth.random_mps(L, 24, seed=11, center=L)
    full = _expand_mps(bonds, sites, L)
    env = D.empty_env()
    for k in range(1, L):
        env = D.left_env_update(env, full[k - 1], k, t, U)
        assert _project_env(env, bonds[k]) < 1e-12
    bonds, sites = synth.random_mps(L, 24, seed=12, center=1)
    full = _expand_mps(bonds, sites, 1)
    env = D.empty_env()
    for k in range(L, 1, -1):
        env = D.right_env_update(env, full[k - 1], k, t, U)
        assert _project_env(env, bonds[k - 1]) < 1e-12


# --------------------------------------------------------------------------
# Dense MPS algebra and TDVP
# --------------------------------------------------------------------------
def test_bond_hopping_decomposition():
    for k in (1, 2, 5):
        o = D.left_channel_ops(k)
        q = D.right_channel_ops(k + 1)
        h = sum(sg * np.kron(o[w][kap], q[w][kap]) for w, sg in ((1, 1), (2, -1)) for kap in range(2))
        assert np.abs((-1) ** k * h + D.two_site_hop(1.0)).max() < 1e-15


def _left_complete(psi, L):
    mps, rest, chi = [None] * L, psi.reshape(1, -1), 1
    for k in range(1, L):
        U_, S, Vh = np.linalg.svd(rest.reshape(chi * 4, -1), full_matrices=False)
        mps[k - 1] = U_.reshape(chi, 4, -1)
        rest, chi = S[:, None] * Vh, S.size
    mps[L - 1] = rest.reshape(chi, 4, 1)
    return mps


def test_environments_recursive_vs_explicit_and_heff_vs_projection():
    L, t, U = 5, 1.0, 4.0
    rng = np.random.default_rng(0)
    psi = rng.normal(size=4 ** L) + 1j * rng.normal(size=4 ** L)
    psi /= np.linalg.norm(psi)
    right = D.complete_right_canonical(psi, L)
    left = _left_complete(psi, L)
    Rv = [None] * (L + 1)
    Rv[L] = D.empty_env()
    for k in range(L, 1, -1):
        Rv[k - 1] = D.right_env_update(Rv[k], right[k - 1], k, t, U)
        ex = D.right_env_explicit(right[k - 1:], k - 1, L, t, U)
        assert max(np.abs(ex[w] - Rv[k - 1][w]).max() for w in range(3)) < 1e-12
    Lv = [D.empty_env()]
    for k in range(1, L):
        Lv.append(D.left_env_update(Lv[-1], left[k - 1], k, t, U))
        ex = D.left_env_explicit(left[:k], k, t, U)
        assert max(np.abs(ex[w] - Lv[k][w]).max() for w in range(3)) < 1e-12
    H = F.hubbard(L, t, U, symmetric=True)
    for i in range(1, L):
        Phi = D.left_block_basis(left[:i - 1]) if i > 1 else np.ones((1, 1))
        Psi = D.right_block_basis(right[i + 1:]) if i + 1 < L else np.ones((1, 1))
        Th = rng.normal(size=(Phi.shape[1], 4, 4, Psi.shape[0])) + 0j
        a = D.heff2(Lv[i - 1], Rv[i + 1], Th, i, t, U)
        b = D.heff2_projected(H, Phi, Psi, Th)
        assert np.abs(a - b).max() < 1e-12 * max(1.0, np.abs(b).max())


def test_lanczos_expm_matches_scipy():
    rng = np.random.default_rng(2)
    n = 60
    M = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    Hm = (M + M.conj().T) / 2
    v = rng.normal(size=n) + 1j * rng.normal(size=n)
    for tau in (-0.05j, 0.05j, -0.3j):
        w, info = D.lanczos_expm(lambda x: Hm @ x, v, tau, tol=1e-13, maxdim=40)
        ref = scipy.linalg.expm(tau * Hm) @ v
        assert info["converged"]
        assert np.abs(w - ref).max() < 1e-11 * np.linalg.norm(v)


@pytest.mark.parametrize("L,nsteps", [(4, 3), (6, 1)])
def test_complete_basis_tdvp_equals_exact_evolution(L, nsteps):
    t, U, dt = 1.0, 4.0, 0.05
    psi0 = F.neel_state(L)
    mps = D.complete_right_canonical(psi0, L)
    H = F.hubbard(L, t, U, symmetric=True)
    exact = F.evolve(H, psi0, np.arange(nsteps + 1) * dt)
    for n in range(nsteps):
        mps, _ = D.tdvp2_sweep(mps, dt, t, U, tol=1e-13)
        v = D.mps_state(mps)
        assert abs(abs(np.vdot(exact[n + 1], v)) - 1) < 1e-12
        assert np.abs(F.local_expectations(v, L)[0] - F.local_expectations(exact[n + 1], L)[0]).max() < 1e-12


def test_complete_basis_time_reversal():
    L, t, U = 4, 1.0, 4.0
    rng = np.random.default_rng(4)
    psi = rng.normal(size=4 ** L) + 1j * rng.normal(size=4 ** L)
    psi /= np.linalg.norm(psi)
    mps = D.complete_right_canonical(psi, L)
    mps, _ = D.tdvp2_sweep(mps, 0.1, t, U, tol=1e-13)
    mps, _ = D.tdvp2_sweep(mps, -0.1, t, U, tol=1e-13)
    assert abs(abs(np.vdot(psi, D.mps_state(mps))) - 1) < 1e-12


@pytest.mark.parametrize("L,nsteps", [(4, 3), (6, 1)])
def test_complete_basis_one_site_tdvp_equals_exact_evolution(L, nsteps):
    """With complete bond bases the one-site tangent-space projector is the
    identity, so one-site TDVP is exact too."""
    t, U, dt = 1.0, 4.0, 0.05
    psi0 = F.neel_state(L)
    mps = D.complete_right_canonical(psi0, L)
    H = F.hubbard(L, t, U, symmetric=True)
    exact = F.evolve(H, psi0, np.arange(nsteps + 1) * dt)
    for n in range(nsteps):
        mps = D.tdvp1_sweep(mps, dt, t, U, tol=1e-13)
        v = D.mps_state(mps)
        assert abs(abs(np.vdot(exact[n + 1], v)) - 1) < 1e-12
        assert np.abs(F.local_expectations(v, L)[0] - F.local_expectations(exact[n + 1], L)[0]).max() < 1e-12


def test_one_site_tdvp_time_reversal_and_conservation_at_fixed_bond():
    """At a bond dimension below the maximal one (a truncated random state),
    one-site TDVP keeps the norm and the energy exactly (projector splitting
    of a Hermitian generator) and a step of -dt undoes a step of +dt to the
    Krylov tolerance."""
    L, t, U = 6, 1.0, 4.0
    rng = np.random.default_rng(9)
    psi = rng.normal(size=4 ** L) + 1j * rng.normal(size=4 ** L)
    psi /= np.linalg.norm(psi)
    mps = D.complete_right_canonical(psi, L)
    # cut every bond to at most 6 states (SVD truncation from the right, renormalised)
    v = D.mps_state(mps).reshape([4] * L)
    cut = []
    rest = v.reshape(1, -1)
    for k in range(L - 1):
        a = rest.shape[0]
        U_, S, Vh = np.linalg.svd(rest.reshape(a * 4, -1), full_matrices=False)
        keep = min(6, S.size)
        cut.append(U_[:, :keep].reshape(a, 4, keep))
        rest = (S[:keep, None] * Vh[:keep])
    cut.append(rest.reshape(-1, 4, 1))
    # right-canonical form of the truncated chain by LQ steps from the right
    start = list(cut)
    for k in range(L - 1, 0, -1):
        a, _, b = start[k].shape
        Q, Rm = np.linalg.qr(start[k].reshape(a, 4 * b).conj().T)
        start[k] = Q.conj().T.reshape(-1, 4, b)
        start[k - 1] = np.tensordot(start[k - 1], Rm.conj().T, axes=([2], [0]))
    start[0] = start[0] / np.linalg.norm(start[0])
    phi = D.mps_state(start)
    bonds = [m.shape[2] for m in start[:-1]]
    assert max(bonds) == 6 and abs(np.linalg.norm(phi) - 1) < 1e-12
    H = F.hubbard(L, t, U, symmetric=True)
    e0 = np.vdot(phi, H @ phi).real
    fwd = D.tdvp1_sweep(start, 0.1, t, U, tol=1e-14)
    w = D.mps_state(fwd)
    assert [m.shape[2] for m in fwd[:-1]] == bonds
    assert abs(np.linalg.norm(w) - 1) < 1e-12
    assert abs(np.vdot(w, H @ w).real - e0) < 1e-10
    back = D.tdvp1_sweep(fwd, -0.1, t, U, tol=1e-14)
    assert abs(abs(np.vdot(phi, D.mps_state(back))) - 1) < 1e-10


# --------------------------------------------------------------------------
# Paper-printed values
# --------------------------------------------------------------------------
def test_table_s2_bond_dimension_bookkeeping():
    """Supplementary Table S2: sum d = chi_SU(2) = 12288, and the full-state
    dimension sum d (2j+1) = 30842 (the paper's chi ~ 30 000)."""
    rows = np.loadtxt(os.path.join(GOLDEN, "table_s2.txt"), dtype=int)
    assert rows.shape == (32, 3)
    assert rows[:, 2].sum() == 12288
    assert int(np.sum(rows[:, 2] * (rows[:, 1] + 1))) == 30842
    assert np.all((rows[:, 0] - rows[:, 1]) % 2 == 0)      # even left block: q = 2j mod 2
    assert rows[:, 2].max() == 1735                          # d_max


def test_synthetic_profile_shape():
    p = synth.sector_profile(4096, 0)
    assert synth.chi_full(p) == 4096
    ratio = synth.chi_full(p) / synth.chi_su2(p)
    assert 2.3 < ratio < 2.6                                 # the paper's chi ~ 2.4 chi_SU(2)


def test_sector_restricted_block_equals_full_dense():
    """The restricted evaluation of one output block, directly and by
    inclusion-exclusion over three smaller restrictions, equals that block of
    the full dense effective Hamiltonian (checked by expanding the block back)."""
    from oracle import sampled as S
    site, t, U = 3, 1.0, 4.0
    left = synth.sector_profile(40, 71, parity=0)
    right = synth.sector_profile(40, 72, parity=0)
    keys = []
    for ia, (qa, tja, da) in enumerate(left):
        for s1, (q1, t1) in enumerate(R.MULTIPLETS):
            for tjx in range(abs(tja - t1), tja + t1 + 1, 2):
                for s2, (q2, t2) in enumerate(R.MULTIPLETS):
                    for ib, (qb, tjb, db) in enumerate(right):
                        if qa + q1 + q2 == qb and abs(tjx - t2) <= tjb <= tjx + t2:
                            keys.append((ia, s1, tjx, s2, ib))

    def env_keys(bond):
        out = []
        for w, (qw, tjw) in enumerate(R.CHANNELS):
            for ii, (qi, tji, _) in enumerate(bond):
                for io, (qo, tjo, _) in enumerate(bond):
                    if qo == qi + qw and abs(tji - tjw) <= tjo <= tji + tjw:
                        out.append((io, w, ii))
        return out
    lk, rk = env_keys(left), env_keys(right)
    theta = synth.block_data(keys, [(left[k[0]][2], right[k[4]][2]) for k in keys], 5)
    Lenv = synth.block_data(lk, [(left[k[0]][2], left[k[2]][2]) for k in lk], 6)
    Renv = synth.block_data(rk, [(right[k[0]][2], right[k[2]][2]) for k in rk], 7)
    full = D.heff2(R.expand_env(Lenv, left), R.expand_env(Renv, right), R.expand_theta(theta, left, right, site),
                   site, t, U)
    rng = np.random.default_rng(0)
    for j in rng.choice(len(keys), size=6, replace=False):
        key = keys[j]
        blk, _ = S.heff2_block(left, right, Lenv, Renv, theta, key, site, t, U)
        cross = S.heff2_block_cross(left, right, Lenv, Renv, theta, key, site, t, U)
        ia, ib = key[0], key[4]
        ref_blk = np.zeros_like(blk)
        for x in range(left[ia][2]):
            for y in range(right[ib][2]):
                e = np.zeros((left[ia][2], right[ib][2]))
                e[x, y] = 1.0
                tree = R.expand_theta({key: e}, left, right, site)
                ref_blk[x, y] = np.vdot(tree, full)
        assert np.abs(blk - ref_blk).max() < 1e-12 * max(1.0, np.abs(ref_blk).max())
        assert np.abs(cross - ref_blk).max() < 1e-12 * max(1.0, np.abs(ref_blk).max())


def _theta_keys(left, right):
    """Reduced two-site blocks (ia, s1, 2j_x, s2, ib) allowed by the fusion rules."""
    fuse = lambda a, b: range(abs(a - b), a + b + 1, 2)
    keys = []
    for ia, (qa, ja, _) in enumerate(left):
        for s1, (q1, j1) in enumerate(R.MULTIPLETS):
            for jx in fuse(ja, j1):
                for s2, (q2, j2) in enumerate(R.MULTIPLETS):
                    for ib, (qb, jb, _) in enumerate(right):
                        if qa + q1 + q2 == qb and jb in fuse(jx, j2):
                            keys.append((ia, s1, jx, s2, ib))
    return keys


def _kept_labels(Um, row_ops):
    """{(q, tj): number of kept multiplets} of an isometry made of whole multiplets."""
    _, labels = D._multiplet_labels(Um, row_ops)
    out = {}
    for q, tj in labels:
        out[(q, tj)] = out.get((q, tj), 0) + 1
    return {k: v // (k[1] + 1) for k, v in out.items()}


def test_multiplet_truncation_matches_reduced_singular_values():
    """The dense singular values of an expanded symmetric two-site tensor are
    the reduced ones of each coupled sector x divided by sqrt(2j_x+1), each
    (2j_x+1)-fold; the dense truncation on labelled multiplets keeps exactly
    the multiplets that the reduced rule of section S2.4 keeps."""
    left = synth.sector_profile(20, 5, parity=1)
    right = synth.sector_profile(20, 6, parity=1)
    keys = _theta_keys(left, right)
    rng = np.random.default_rng(4)
    blocks = {k: rng.standard_normal((left[k[0]][2], right[k[4]][2]))
              + 1j * rng.standard_normal((left[k[0]][2], right[k[4]][2])) for k in keys}
    Th = R.expand_theta(blocks, left, right, 2)
    a, b = Th.shape[0], Th.shape[-1]
    M = Th.reshape(a * 4, 4 * b)
    sv = R.sector_singular_values(blocks, left, right)
    # the reduced values against an SVD of each sector matrix assembled here by hand
    for (qx, jx), s in sv.items():
        ks = [k for k in keys if left[k[0]][0] + R.MULTIPLETS[k[1]][0] == qx and k[2] == jx]
        rows = sorted({(k[0], k[1]) for k in ks})
        cols = sorted({(k[3], k[4]) for k in ks})
        ro = np.cumsum([0] + [left[r[0]][2] for r in rows])
        co = np.cumsum([0] + [right[c[1]][2] for c in cols])
        Mx = np.zeros((ro[-1], co[-1]), complex)
        for k in ks:
            i, j = rows.index((k[0], k[1])), cols.index((k[3], k[4]))
            Mx[ro[i]:ro[i + 1], co[j]:co[j + 1]] = blocks[k]
        ref = np.linalg.svd(Mx, compute_uv=False)
        assert s.shape == ref.shape and np.allclose(s, ref, rtol=0, atol=1e-12 * ref[0])
    full = np.sort(np.concatenate([np.repeat(s / np.sqrt(jx + 1), jx + 1) for (qx, jx), s in sv.items()]))[::-1]
    dense = np.linalg.svd(M, compute_uv=False)
    assert np.allclose(dense[:full.size], full, rtol=0, atol=1e-12 * full[0])
    assert np.all(dense[full.size:] < 1e-12 * full[0])
    ops = R.row_quantum_ops(left, 2)
    W = np.sum(dense ** 2)
    for eps, cap in ((1e-2, 10 ** 9), (0.0, 40), (1e-3, 60), (0.2, 25)):
        kept, disc_r = R.truncate_multiplets(sv, eps, cap)
        Um, S, Vh, disc = D._svd_split(M, False, eps, cap, multiplets=True, row_ops=ops)
        assert S.size == sum(n * (x[1] + 1) for x, n in kept.items())
        assert abs(disc - disc_r) < 1e-12
        assert _kept_labels(Um, ops) == {x: n for x, n in kept.items() if n}
        assert abs(np.sum(S ** 2) - W) < 1e-10 * W
        # the kept part is the projection of M on the kept left singular space
        assert np.abs(Um @ (np.diag(S) @ Vh) * np.sqrt(1 - disc) - Um @ (Um.conj().T @ M)).max() < 1e-12 * dense[0]


def test_tied_multiplets_follow_the_tie_rule():
    """Two multiplets of different sectors with equal full-state singular
    values: the one with the smaller (q, 2j) comes first, so a cap that fits
    only one keeps that one, in the reduced rule and in the dense truncation
    of the expanded tensor alike."""
    left = synth.sector_profile(20, 5, parity=1)
    right = synth.sector_profile(20, 6, parity=1)
    site = 2
    mats = R.sector_matrices({}, left, right)
    rng = np.random.default_rng(11)
    xs = sorted(mats)
    big = [x for x in xs if min(mats[x][0].shape) >= 2]
    # the tied pair: a (q, 0) singlet and a (q', 2) triplet sector, q < q'
    x_lo = min(x for x in big if x[1] == 2)
    x_hi = min(x for x in big if x[1] == 0 and x[0] > x_lo[0])
    blocks = {}
    for x in xs:
        Mx, rows, cols = mats[x]
        r = min(Mx.shape)
        s = np.sort(rng.uniform(0.05, 0.5, r))[::-1] * np.sqrt(x[1] + 1)
        if x in (x_lo, x_hi):
            s[0] = 2.0 * np.sqrt(x[1] + 1)          # equal full-state value 2.0, above all others
        Ux, _ = np.linalg.qr(rng.standard_normal((Mx.shape[0], r)) + 1j * rng.standard_normal((Mx.shape[0], r)))
        Vx, _ = np.linalg.qr(rng.standard_normal((Mx.shape[1], r)) + 1j * rng.standard_normal((Mx.shape[1], r)))
        Mx = (Ux * s) @ Vx.conj().T
        ro = np.cumsum([0] + [left[a][2] for a, _ in rows])
        co = np.cumsum([0] + [right[bb][2] for _, bb in cols])
        for i, (ia, s1) in enumerate(rows):
            for j, (s2, ib) in enumerate(cols):
                # every (row partner, column partner) pair of a sector is an allowed block
                blocks[(ia, s1, x[1], s2, ib)] = Mx[ro[i]:ro[i + 1], co[j]:co[j + 1]]
    assert set(blocks) == set(map(tuple, _theta_keys(left, right)))
    svals = R.sector_singular_values(blocks, left, right)
    assert abs(svals[x_lo][0] / np.sqrt(x_lo[1] + 1) - svals[x_hi][0]) < 1e-12
    Th = R.expand_theta(blocks, left, right, site)
    M = Th.reshape(Th.shape[0] * 4, -1)
    ops = R.row_quantum_ops(left, site)
    first = min(x_lo, x_hi)
    for cap in (1, 3, 4):
        kept, _ = R.truncate_multiplets(svals, 0.0, cap)
        Um, S, Vh, _ = D._svd_split(M, False, 0.0, cap, multiplets=True, row_ops=ops)
        assert kept[first] == 1
        assert _kept_labels(Um, ops) == {x: n for x, n in kept.items() if n}
    kept1, _ = R.truncate_multiplets(svals, 0.0, 1)
    assert {x: n for x, n in kept1.items() if n} == {first: 1}


# ---- abelian U(1) x U(1) expansion (oracle.abelian) --------------------------
def _u1_chain(L, seed, chi):
    """Bonds of a U(1) x U(1) chain (vacuum, profiles, total (N, 2Sz) = (L, 0))
    and random blocks for every allowed (a, s, b) key of each site."""
    from oracle import abelian as A
    bonds = [[(0, 0, 1)]] + [synth.u1_profile(chi, seed + k, k, window=2) for k in range(1, L)] + [[(0, L, 1)]]
    sites = []
    for k in range(1, L + 1):
        left, right = bonds[k - 1], bonds[k]
        keys = [(a, s, b) for a in range(len(left)) for s in range(4) for b in range(len(right))
                if left[a][1] + A.LOCAL_N[s] == right[b][1] and left[a][0] + A.LOCAL_SZ2[s] == right[b][0]]
        dims = [(left[a][2], right[b][2]) for a, _, b in keys]
        sites.append(synth.block_data(keys, dims, seed + 100 + k))
    return bonds, sites


def test_abelian_expansion_has_the_labelled_charges():
    """A random U(1) x U(1) chain expanded by oracle.abelian and contracted
    to a state vector is an eigenvector of the total particle number (L) and
    of 2 S^z (0), built from the Jordan-Wigner operators of oracle.fermions;
    and the left block of every bond k, contracted separately, has on each
    sector's columns exactly that sector's (N, 2S^z)."""
    from oracle import abelian as A
    L = 6
    bonds, sites = _u1_chain(L, 400, 9)
    full = [A.expand_site(sites[k - 1], bonds[k - 1], bonds[k]) for k in range(1, L + 1)]
    psi = D.mps_state(full)
    assert np.linalg.norm(psi) > 1e-3
    c = {(i, s): F.annihilator(i, s, L) for i in range(1, L + 1) for s in (0, 1)}
    N = sum(c[(i, s)].T @ c[(i, s)] for i in range(1, L + 1) for s in (0, 1))
    Sz2 = sum(c[(i, 0)].T @ c[(i, 0)] - c[(i, 1)].T @ c[(i, 1)] for i in range(1, L + 1))
    assert np.abs(N @ psi - L * psi).max() < 1e-12 * np.abs(psi).max()
    assert np.abs(Sz2 @ psi).max() < 1e-12 * np.abs(psi).max()
    for k in range(1, L):
        Phi = D.left_block_basis(full[:k])            # [(s_1..s_k), b]
        ck = {(i, s): F.annihilator(i, s, k) for i in range(1, k + 1) for s in (0, 1)}
        Nk = sum(ck[(i, s)].T @ ck[(i, s)] for i in range(1, k + 1) for s in (0, 1)).toarray()
        Sk = sum(ck[(i, 0)].T @ ck[(i, 0)] - ck[(i, 1)].T @ ck[(i, 1)] for i in range(1, k + 1)).toarray()
        off, _ = A.offsets(bonds[k])
        for (sz2, n, d), o in zip(bonds[k], off):
            cols = Phi[:, o:o + d]
            assert np.abs(Nk @ cols - n * cols).max() < 1e-12 * max(np.abs(cols).max(), 1.0)
            assert np.abs(Sk @ cols - sz2 * cols).max() < 1e-12 * max(np.abs(cols).max(), 1.0)


def test_abelian_environments_live_on_their_channel_blocks():
    """Environments of the expanded chain, built by the oracle's dense
    updates, are zero outside the blocks the abelian channel labels allow:
    cutting them into oracle.abelian's (out, w, in) blocks and expanding
    again reproduces them exactly, left and right, every channel."""
    from oracle import abelian as A
    L, t, U = 6, 1.0, 4.0
    bonds, sites = _u1_chain(L, 500, 10)
    full = [A.expand_site(sites[k - 1], bonds[k - 1], bonds[k]) for k in range(1, L + 1)]
    dw = {0: (0, 0), 1: (1, 1), 2: (-1, 1), 3: (1, -1), 4: (-1, -1)}   # (dN, d2Sz) of each channel
    def keys(bond):
        return [(io, w, ii) for w in range(5) for ii in range(len(bond)) for io in range(len(bond))
                if bond[io][1] == bond[ii][1] + dw[w][0] and bond[io][0] == bond[ii][0] + dw[w][1]]
    Lf = D.empty_env()
    for k in range(1, L):
        Lf = D.left_env_update(Lf, full[k - 1], k, t, U)
        back = A.expand_env(A.restrict_env(Lf, bonds[k], keys(bonds[k])), bonds[k])
        assert all(np.array_equal(back[w], Lf[w]) for w in range(3))
        assert max(np.abs(Lf[w]).max() for w in (1, 2)) > 0
    Rf = D.empty_env()
    for k in range(L, 1, -1):
        Rf = D.right_env_update(Rf, full[k - 1], k, t, U)
        back = A.expand_env(A.restrict_env(Rf, bonds[k - 1], keys(bonds[k - 1])), bonds[k - 1])
        assert all(np.array_equal(back[w], Rf[w]) for w in range(3))
