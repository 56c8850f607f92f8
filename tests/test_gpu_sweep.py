"""Two-site TDVP sweeps on the GPU against exact evolution.

With every bond at its full symmetric dimension (zero-weight directions
kept) two-site TDVP is exact, so the L = 8 Neel quench (U/J = 4,
dt = 0.05) must follow the exact state-vector evolution of Eq. (1) to the
Krylov tolerance."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2606_04771_amd as T
from oracle import dense as D
from oracle import fermions as F
from oracle import reduced as R
from tests._harness import unpack, theta_dict

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    c = T.Context(0)
    yield c
    c.close()


def mps_state(mps, L):
    """Expand the library MPS (centre C1 on site 1, B elsewhere) with the
    oracle's conventions and contract it to a state vector."""
    bonds = [mps.bond(k) for k in range(L + 1)]
    full = []
    for k in range(1, L + 1):
        keys, offs, data = mps.site(k)
        dims = [(bonds[k - 1][kk[0]][2], bonds[k][kk[2]][2]) for kk in keys]
        blocks = theta_dict(keys, unpack(data, offs, dims))
        full.append(R.expand_site("C" if k == 1 else "B", blocks, bonds[k - 1], bonds[k], k))
    return D.mps_state(full)


def test_neel_mps_is_the_neel_state(ctx):
    L = 6
    for complete in (False, True):
        mps = T.MPS.neel(ctx, T.Model(L, 1.0, 4.0), complete=complete)
        psi = mps_state(mps, L)
        ref = F.neel_state(L)
        assert abs(abs(np.vdot(ref, psi)) - 1) < 1e-14
        assert abs(np.linalg.norm(psi) - 1) < 1e-14
        sz, docc, n2 = mps.measure()
        assert np.abs(sz - 0.5 * (-1.0) ** np.arange(L)).max() < 1e-14   # site 1 up
        assert np.abs(docc).max() < 1e-14
        assert abs(n2 - 1) < 1e-14
        mps.close()


def test_complete_basis_sweeps_follow_exact_evolution_L8(ctx):
    """Config: L = 8, U/J = 4, half filling, Neel start, complete bases,
    dt = 0.05; compared with the 4^8 state vector.  The Lanczos tolerance is
    1e-14 so that ~1000 exponentials stay within 1e-10 (at 1e-12 the drift of
    the densities reaches 2.4e-10 by t = 2, the accumulated tolerance)."""
    L, t, U, dt, nsteps = 8, 1.0, 4.0, 0.05, 40
    model = T.Model(L, t, U)
    mps = T.MPS.neel(ctx, model, complete=True)
    H = F.hubbard(L, t, U)            # Eq. (1) form: differs by a global phase only
    psi0 = F.neel_state(L)
    times = np.arange(nsteps + 1) * dt
    exact = F.evolve(H, psi0, times)
    worst_n = worst_ov = 0.0
    for n in range(1, nsteps + 1):
        info = mps.sweep(dt, keep_all=True, krylov_tol=1e-14, krylov_maxdim=50)
        assert info["nonconverged"] == 0
        if n % 10 == 0 or n == 1:
            psi = mps_state(mps, L)
            ov = abs(np.vdot(exact[n], psi))
            nu, nd, dd = F.local_expectations(psi, L)
            nu0, nd0, dd0 = F.local_expectations(exact[n], L)
            worst_ov = max(worst_ov, abs(1 - ov))
            worst_n = max(worst_n, np.abs(nu - nu0).max(), np.abs(dd - dd0).max())
            # the library's own observables against the exact ones
            sz, docc, n2 = mps.measure()
            worst_n = max(worst_n, np.abs(sz - 0.5 * (nu0 - nd0)).max(), np.abs(docc - dd0).max(), abs(n2 - 1))
            print(f"t={n * dt:.2f} 1-|ov|={1 - ov:.2e} max|dn|={np.abs(nu - nu0).max():.2e} "
                  f"chi={info['max_chi']} krylov={info['krylov_iters']}", flush=True)
    mps.close()
    assert worst_ov < 1e-10
    assert worst_n < 1e-10


def test_truncated_sweep_invariants(ctx):
    """Finite bond dimension: norm 1, <n_i> = 1, S^z = 0 and the discarded
    weight bound hold after every sweep."""
    L, dt = 8, 0.05
    mps = T.MPS.neel(ctx, T.Model(L, 1.0, 4.0), complete=False)
    for n in range(8):
        info = mps.sweep(dt, eps_tol=1e-6, chi_cap=24, keep_all=False)
        assert info["max_chi"] <= 24
        psi = mps_state(mps, L)
        assert abs(np.linalg.norm(psi) - 1) < 1e-12
        nu, nd, dd = F.local_expectations(psi, L)
        assert np.abs(nu + nd - 1).max() < 1e-10
        assert abs(np.sum(nu - nd)) < 1e-10
        sz, docc, n2 = mps.measure()
        assert np.abs(sz - 0.5 * (nu - nd)).max() < 1e-12
        assert np.abs(docc - dd).max() < 1e-12
        assert abs(n2 - 1) < 1e-12
    mps.close()
