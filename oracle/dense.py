"""Dense MPS algebra for the two-site TDVP hot path.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything works on full tensors in the Jordan-Wigner basis of
``oracle.fermions``: site tensors ``M[chi_left, 4, chi_right]``, two-site
tensors ``Th[chi_left, 4, 4, chi_right]``, and environments stored per channel
as ``{w: E[chi, n_kappa, chi]}`` (w = 0 'H', 1 'D+', 2 'D-'; n_kappa = 1, 2, 2),
the same layout ``oracle.reduced.expand_env`` produces.

Definitions (supplementary section S2.2: TDVP merges one or two sites,
exponentiates the effective Hamiltonian of that block with a Krylov method
and sweeps; section S2.3: the dominant work is the environment updates and
the Krylov exponentials):

* Left environment at bond k (block of sites 1..k with basis |Phi>):
     'H'  : <Phi'| H_block |Phi>        (H restricted to sites 1..k)
     'D+' : <Phi'| O^{D+}_kappa |Phi>,  'D-' likewise,
  with the edge operators of ``left_channel_ops(k)`` acting on site k.
* Right environment at bond k (block of sites k+1..L with basis |Psi>):
     'H'  : <Psi'| H_block |Psi>,  'D+'/'D-': <Psi'| Q^{w}_kappa |Psi>
  with the operators of ``right_channel_ops(k+1)`` acting on site k+1.
* The hopping across a bond (k, k+1) of Eq. (1) equals
     (-1)^k sum_kappa [ O^{D+}_kappa(k) Q^{D+}_kappa(k+1) - O^{D-}_kappa(k) Q^{D-}_kappa(k+1) ]
  (checked against the Jordan-Wigner operators in the tests).
* The effective Hamiltonian of sites (i, i+1) acting on Th is the projection
  P^dag H P with P = |Phi_{i-1}> x 1 x 1 x |Psi_{i+1}>; written with the
  environments it is the sum of the terms in ``heff2``.

The interaction is the particle-hole symmetric U (n_up - 1/2)(n_dn - 1/2),
the form for which the pseudospin SU(2) of section S2.1 is exact.
"""
import functools

import numpy as np
import scipy.linalg

from .fermions import A_UP, A_DN, PARITY, N_UP, N_DN, EYE4, hubbard

TJ_W = [0, 1, 1]


def _es(spec, *ops):
    """einsum with numpy's pairwise contraction order (same result, BLAS speed)."""
    return np.einsum(spec, *ops, optimize=True)


def left_channel_ops(k):
    """Edge operators of a left block whose last site is k (1-based):
    {w: [op_kappa=+1/2, op_kappa=-1/2]} (w = 1 'D+', 2 'D-').
    They are the pseudospin doublets D+ = (c+_up, (-1)^k c_dn) and
    D- = (c+_dn, -(-1)^k c_up) of site k times the site parity."""
    sg = (-1.0) ** k
    return {1: [A_UP.T @ PARITY, sg * A_DN @ PARITY],
            2: [A_DN.T @ PARITY, -sg * A_UP @ PARITY]}


def right_channel_ops(k):
    """Partner operators on site k for a hopping that enters from the left:
    Q^{D+}_kappa = eps(kappa) [D-]_{-kappa},  Q^{D-}_kappa = eps(kappa) [D+]_{-kappa},
    eps(+1/2) = +1, eps(-1/2) = -1, with the doublets of site k."""
    sg = (-1.0) ** k
    return {1: [-sg * A_UP, -A_DN.T],
            2: [sg * A_DN, -A_UP.T]}


def onsite(U):
    """U (n_up - 1/2)(n_dn - 1/2) on one site."""
    return U * (N_UP - 0.5 * EYE4) @ (N_DN - 0.5 * EYE4)


@functools.lru_cache(maxsize=None)
def two_site_hop(t):
    """-t sum_s (c+_1s c_2s + h.c.) on a two-site chain, as a 16x16 matrix in
    the local basis (site 1 slow).  Taken from the Jordan-Wigner Hamiltonian
    of a two-site chain with U = 0."""
    return hubbard(2, t=t, U=0.0).toarray()


# ----------------------------------------------------------------------------
# MPS <-> state vector, explicit block bases
# ----------------------------------------------------------------------------
def mps_state(mps):
    """Contract a dense MPS [M_1 .. M_L] (boundary bonds of dimension 1) to a
    state vector of length 4^L."""
    v = mps[0]
    for M in mps[1:]:
        v = np.tensordot(v, M, axes=([v.ndim - 1], [0]))
    return v.reshape(-1)


def left_block_basis(sites):
    """Matrix Phi[(s_1..s_k), b] of the left block states defined by the
    tensors of sites 1..k (first bond of dimension 1)."""
    v = sites[0][0]                      # [4, chi_1]
    for M in sites[1:]:
        v = np.tensordot(v, M, axes=([v.ndim - 1], [0]))
    return v.reshape(-1, v.shape[-1])


def right_block_basis(sites):
    """Matrix Psi[b, (s_{k+1}..s_L)] of the right block states defined by the
    tensors of sites k+1..L (last bond of dimension 1)."""
    v = sites[-1][..., 0]                # [chi, 4]
    for M in reversed(sites[:-1]):
        v = np.tensordot(M, v, axes=([2], [0]))
    return v.reshape(v.shape[0], -1)


def block_hamiltonian(n, t, U):
    """Hubbard Hamiltonian (symmetric interaction) of an isolated block of n
    sites, dense."""
    if n == 0:
        return np.zeros((1, 1))
    return hubbard(n, t=t, U=U, symmetric=True).toarray()


def _embed(op, pos, n):
    """Operator acting on the pos-th (1-based) site of an n-site block."""
    return np.kron(np.kron(np.eye(4 ** (pos - 1)), op), np.eye(4 ** (n - pos)))


def left_env_explicit(sites, k, t, U):
    """Left environment at bond k computed from the explicit block basis
    (sites = tensors of sites 1..k, k >= 1)."""
    Phi = left_block_basis(sites)
    Hb = block_hamiltonian(k, t, U)
    env = {0: (Phi.conj().T @ Hb @ Phi)[:, None, :]}
    ops = left_channel_ops(k)
    for w in (1, 2):
        env[w] = np.stack([Phi.conj().T @ _embed(op, k, k) @ Phi for op in ops[w]], axis=1)
    return env


def right_env_explicit(sites, k, L, t, U):
    """Right environment at bond k (block of sites k+1..L) from the explicit
    block basis (sites = tensors of sites k+1..L)."""
    Psi = right_block_basis(sites)
    n = L - k
    Hb = block_hamiltonian(n, t, U)
    env = {0: (Psi.conj() @ Hb @ Psi.T)[:, None, :]}
    ops = right_channel_ops(k + 1)
    for w in (1, 2):
        env[w] = np.stack([Psi.conj() @ _embed(op, 1, n) @ Psi.T for op in ops[w]], axis=1)
    return env


def empty_env():
    """Environment of an empty block (bond of dimension 1)."""
    return {0: np.zeros((1, 1, 1), complex), 1: np.zeros((1, 2, 1), complex),
            2: np.zeros((1, 2, 1), complex)}


# ----------------------------------------------------------------------------
# environment updates (recursive definition)
# ----------------------------------------------------------------------------
def left_env_update(env, A, k, t, U):
    """Left environment at bond k from the one at bond k-1 and the
    left-canonical tensor A of site k:
      H'   = A^dag (H x 1 + 1 x onsite_k + hop(k-1, k)) A
      D'_w = A^dag (1 x O^w_kappa(k)) A
    where hop(k-1,k) couples the old edge operators to the partners on site k."""
    Ac = A.conj()
    # H part: old block Hamiltonian carried through
    X = _es("xy,ysb->xsb", env[0][:, 0, :], A)
    Hn = _es("xsc,xsb->cb", Ac, X)
    # on-site term of site k
    Hn = Hn + _es("xsc,st,xtb->cb", Ac, onsite(U), A)
    # hopping across (k-1, k)
    if k > 1:
        sg = (-1.0) ** (k - 1)
        qops = right_channel_ops(k)
        for w, sign in ((1, 1.0), (2, -1.0)):
            for kap in range(2):
                Y = _es("xy,st,ytb->xsb", env[w][:, kap, :], qops[w][kap], A)
                Hn = Hn + (-t) * sg * sign * _es("xsc,xsb->cb", Ac, Y)
    out = {0: Hn[:, None, :]}
    ops = left_channel_ops(k)
    for w in (1, 2):
        out[w] = np.stack([_es("xsc,st,xtb->cb", Ac, op, A) for op in ops[w]], axis=1)
    return out


def right_env_update(env, B, k, t, U):
    """Right environment at bond k-1 from the one at bond k and the
    right-canonical tensor B of site k (B[chi_{k-1}, 4, chi_k]):
      H'   = B (H x 1 + onsite_k x 1 + hop(k, k+1)) B^dag
      D'_w = B (Q^w_kappa(k) x 1) B^dag
    written with <Psi'| . |Psi> ordering: E'[x', x] = sum conj(B[x',..]) (.) B[x,..]."""
    Bc = B.conj()
    X = _es("xsb,yb->xsy", B, env[0][:, 0, :])        # [x, s, b']
    Hn = _es("zsy,xsy->zx", Bc, X)
    Hn = Hn + _es("zsb,st,xtb->zx", Bc, onsite(U), B)
    sg = (-1.0) ** k
    oops = left_channel_ops(k)
    for w, sign in ((1, 1.0), (2, -1.0)):
        for kap in range(2):
            Y = _es("st,xtb,yb->xsy", oops[w][kap], B, env[w][:, kap, :])
            Hn = Hn + (-t) * sg * sign * _es("zsy,xsy->zx", Bc, Y)
    out = {0: Hn[:, None, :]}
    qops = right_channel_ops(k)
    for w in (1, 2):
        out[w] = np.stack([_es("zsb,st,xtb->zx", Bc, op, B) for op in qops[w]], axis=1)
    return out


# ----------------------------------------------------------------------------
# effective Hamiltonians
# ----------------------------------------------------------------------------
def heff2(Lenv, Renv, Th, i, t, U):
    """Effective Hamiltonian of sites (i, i+1) applied to Th[a, s1, s2, b].
    Lenv: left environment at bond i-1; Renv: right environment at bond i+1."""
    out = _es("xy,ystb->xstb", Lenv[0][:, 0, :], Th)
    out += _es("zb,xstb->xstz", Renv[0][:, 0, :], Th)
    hU = onsite(U)
    out += _es("su,xutb->xstb", hU, Th)
    out += _es("tu,xsub->xstb", hU, Th)
    h2 = two_site_hop(t).reshape(4, 4, 4, 4)
    out += _es("stuv,xuvb->xstb", h2, Th)
    # hopping across (i-1, i): left edge operators x partners on site i
    sgl = (-1.0) ** (i - 1)
    q = right_channel_ops(i)
    for w, sign in ((1, 1.0), (2, -1.0)):
        for kap in range(2):
            out += (-t) * sgl * sign * _es("xy,su,yutb->xstb", Lenv[w][:, kap, :],
                                                 q[w][kap], Th)
    # hopping across (i+1, i+2): operators on site i+1 x right edge partners
    sgr = (-1.0) ** (i + 1)
    o = left_channel_ops(i + 1)
    for w, sign in ((1, 1.0), (2, -1.0)):
        for kap in range(2):
            out += (-t) * sgr * sign * _es("tu,zb,xsub->xstz", o[w][kap],
                                                 Renv[w][:, kap, :], Th)
    return out


def heff1(Lenv, Renv, C, k, t, U):
    """Effective Hamiltonian of site k applied to C[a, s, b].
    Lenv: left environment at bond k-1; Renv: right environment at bond k."""
    out = _es("xy,ysb->xsb", Lenv[0][:, 0, :], C)
    out += _es("zb,xsb->xsz", Renv[0][:, 0, :], C)
    out += _es("su,xub->xsb", onsite(U), C)
    sgl = (-1.0) ** (k - 1)
    q = right_channel_ops(k)
    for w, sign in ((1, 1.0), (2, -1.0)):
        for kap in range(2):
            out += (-t) * sgl * sign * _es("xy,su,yub->xsb", Lenv[w][:, kap, :], q[w][kap], C)
    sgr = (-1.0) ** k
    o = left_channel_ops(k)
    for w, sign in ((1, 1.0), (2, -1.0)):
        for kap in range(2):
            out += (-t) * sgr * sign * _es("su,zb,xub->xsz", o[w][kap], Renv[w][:, kap, :], C)
    return out


def heff2_projected(H, Phi, Psi, Th):
    """Plain definition P^dag H P Th with P = Phi x 1 x 1 x Psi^T
    (Phi: left block basis [4^(i-1), chi], Psi: right block basis [chi, 4^(L-i-1)])."""
    nl, a = Phi.shape
    b, nr = Psi.shape
    P = np.kron(np.kron(Phi, np.eye(16)), Psi.T)          # [4^L, a*16*b]
    return (P.conj().T @ (H @ (P @ Th.reshape(-1)))).reshape(Th.shape)


# ----------------------------------------------------------------------------
# Krylov exponential
# ----------------------------------------------------------------------------
def lanczos_expm(apply, v, tau, tol=1e-12, maxdim=40):
    """exp(tau H) v for Hermitian H given as ``apply``.

    Lanczos with full re-orthogonalisation (two classical Gram-Schmidt
    passes).  After each new vector the Krylov approximation
    y = |v| exp(tau T_m) e_1 is formed and the iteration stops when the
    a-posteriori estimate beta_m |y_m| <= tol |v| (the adaptive-dimension rule
    cited by the paper in section S2.2), on a happy breakdown, or at maxdim.
    Returns (w, info) with info = {'iters', 'err', 'converged'}."""
    shape = v.shape
    nrm = np.linalg.norm(v)
    if nrm == 0.0:
        return v.copy(), {"iters": 0, "err": 0.0, "converged": True}
    V = [v.reshape(-1) / nrm]
    alpha, beta = [], []
    err = np.inf
    for m in range(1, maxdim + 1):
        w = apply(V[-1].reshape(shape)).reshape(-1)
        a = np.vdot(V[-1], w).real
        alpha.append(a)
        w = w - a * V[-1] - (beta[-1] * V[-2] if m > 1 else 0.0)
        for _ in range(2):
            Vm = np.array(V)
            w = w - Vm.T @ (Vm.conj() @ w)
        b = np.linalg.norm(w)
        T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
        y = scipy.linalg.expm(tau * T)[:, 0] * nrm
        err = b * abs(y[-1])
        if b < 1e-14 * nrm or err <= tol * nrm or m == maxdim:
            out = np.array(V).T @ y
            return out.reshape(shape), {"iters": m, "err": float(err),
                                        "converged": bool(b < 1e-14 * nrm or err <= tol * nrm)}
        beta.append(b)
        V.append(w / b)


# ----------------------------------------------------------------------------
# complete MPS and the two-site TDVP sweep
# ----------------------------------------------------------------------------
def complete_right_canonical(psi, L):
    """Right-canonical MPS [C_1, B_2, ..., B_L] of a state vector with every
    bond at its maximal dimension min(4^k, 4^(L-k)): every singular value is
    kept, zero ones included, so the bases are complete."""
    mps = [None] * L
    rest = psi.reshape(-1, 1)            # [4^L, 1]
    chi_r = 1
    for k in range(L, 1, -1):
        M = rest.reshape(-1, 4 * chi_r)  # [4^(k-1), 4 chi_r]
        U_, S, Vh = np.linalg.svd(M, full_matrices=False)
        chi = S.size
        mps[k - 1] = Vh.reshape(chi, 4, chi_r)
        rest = U_ * S
        chi_r = chi
    mps[0] = rest.reshape(1, 4, chi_r)
    return mps


def _multiplet_labels(U, row_ops):
    """(q, tj) of the left singular vectors U of one group of equal singular
    values: U rotated to simultaneous eigenvectors of 2 S^z and T^2 of the
    rows (row_ops = (Sz2, T2)).  Returns (R, labels), U R being the rotated
    vectors and labels[c] = (q, tj) of column c."""
    Sz2, T2 = row_ops
    qv, Y = np.linalg.eigh(U.conj().T @ (Sz2 @ U))
    R, labels = [], []
    qr = np.rint(qv).astype(int)
    for q in sorted(set(qr)):
        Yq = Y[:, qr == q]
        tv, Z = np.linalg.eigh(Yq.conj().T @ (U.conj().T @ (T2 @ (U @ Yq))))
        tj = np.rint(np.sqrt(np.maximum(4.0 * tv + 1.0, 0.0)) - 1.0).astype(int)
        for v in sorted(set(tj)):
            R.append(Yq @ Z[:, tj == v])
            labels += [(int(q), int(v))] * int(np.sum(tj == v))
    return np.concatenate(R, axis=1), labels


def _svd_split(M, keep_all, eps_tol, chi_cap, multiplets=False, row_ops=None):
    """SVD of the merged two-site matrix with the truncation of supplementary
    section S2: singular values are dropped from the smallest while the
    discarded squared weight stays within eps_tol of the total and while more
    than chi_cap values remain (at least one is kept); the kept values are
    renormalised to the original norm.

    With ``multiplets`` the values are handled as whole multiplets of the
    pseudospin symmetry: a group of (numerically) equal values is split by
    the quantum numbers (q, tj) of the left part (``row_ops`` = (2 S^z, T^2)
    on the rows), each (q, tj) part into multiplets of tj + 1 values; the
    multiplets are ordered by value (descending), ties by q, then tj
    (ascending), and kept or dropped whole, the cap stopping at the first
    multiplet that does not fit."""
    U_, S, Vh = np.linalg.svd(M, full_matrices=False)
    if keep_all:
        return U_, S, Vh, 0.0
    w = S ** 2
    tot = w.sum()
    if not multiplets:
        keep = S.size
        disc = 0.0
        while keep > 1 and (disc + w[keep - 1] <= eps_tol * tot or keep > chi_cap):
            disc += w[keep - 1]
            keep -= 1
        S = S[:keep] / np.sqrt(1.0 - disc / tot) if tot > 0 else S[:keep]
        return U_[:, :keep], S, Vh[:keep], disc / tot if tot > 0 else 0.0
    # groups of equal values, each split into labelled multiplets
    tolg = 1e-9 * (S[0] if S.size else 0.0)
    mults = []        # (value, q, tj, columns of U, rows of Vh)
    start = 0
    for i in range(1, S.size + 1):
        if i < S.size and S[i - 1] - S[i] <= tolg:
            continue
        Ug, Vg = U_[:, start:i], Vh[start:i]
        R, labels = _multiplet_labels(Ug, row_ops)
        Ur, Vr = Ug @ R, R.conj().T @ Vg
        c = 0
        while c < len(labels):
            q, tj = labels[c]
            mults.append((S[start], q, tj, Ur[:, c:c + tj + 1], Vr[c:c + tj + 1], S[start:start + tj + 1]))
            c += tj + 1
        start = i
    mults.sort(key=lambda m: (-m[0], m[1], m[2]))
    mw = [np.sum(m[5] ** 2) for m in mults]
    keep, tail = len(mults), 0.0
    while keep > 1 and tail + mw[keep - 1] <= eps_tol * tot:
        tail += mw[keep - 1]
        keep -= 1
    n, p = 0, 0
    while p < keep and (p == 0 or n + mults[p][2] + 1 <= chi_cap):
        n += mults[p][2] + 1
        p += 1
    disc = tot - sum(mw[:p])
    Uk = np.concatenate([m[3] for m in mults[:p]], axis=1)
    Vk = np.concatenate([m[4] for m in mults[:p]], axis=0)
    Sk = np.concatenate([np.full(m[2] + 1, m[0]) for m in mults[:p]])
    Sk = Sk / np.sqrt(1.0 - disc / tot) if tot > 0 else Sk
    return Uk, Sk, Vk, disc / tot if tot > 0 else 0.0


_BLOCK_OPS = {}


def _block_ops(n):
    """T+, Tz and 2 S^z of a block of n sites (cached: they depend on n only)."""
    if n not in _BLOCK_OPS:
        from .fermions import pseudospin
        Tp, _, Tz = pseudospin(n)
        idx = np.arange(4 ** n)
        sz = np.zeros(4 ** n)
        for k in range(n):
            s = (idx // 4 ** (n - 1 - k)) % 4
            sz += (s == 1).astype(float) - (s == 2).astype(float)
        _BLOCK_OPS[n] = (Tp, Tz, sz)
    return _BLOCK_OPS[n]


def left_row_ops(mps, i):
    """(2 S^z, T^2) of sites 1..i on the row space (left bond index, state of
    site i) of the two-site tensor at sites (i, i+1), from the left-canonical
    tensors mps[0..i-2] (their left block basis Phi) and the fermion
    operators: Phi^dag O_block Phi (x) 1 + 1 (x) o_site."""
    from .fermions import A_UP, A_DN
    nu, nd = A_UP.T @ A_UP, A_DN.T @ A_DN
    tp = (-1.0) ** i * (A_UP.T @ A_DN.T)
    tz = 0.5 * (nu + nd - np.eye(4))
    if i == 1:
        Jp, Jz, Q = np.zeros((1, 1)), np.zeros((1, 1)), np.zeros((1, 1))
    else:
        Phi = left_block_basis(mps[:i - 1])
        Tp_b, Tz_b, sz = _block_ops(i - 1)
        Jp = Phi.conj().T @ (Tp_b @ Phi)
        Jz = Phi.conj().T @ (Tz_b @ Phi)
        Q = Phi.conj().T @ (sz[:, None] * Phi)
    a = Jp.shape[0]
    I4, Ia = np.eye(4), np.eye(a)
    Tp = np.kron(Jp, I4) + np.kron(Ia, tp)
    Tz = np.kron(Jz, I4) + np.kron(Ia, tz)
    T2 = Tp @ Tp.conj().T + Tz @ Tz - Tz
    return np.kron(Q, I4) + np.kron(Ia, nu - nd), T2


def tdvp2_sweep(mps, dt, t, U, tol=1e-12, maxdim=40, keep_all=True, eps_tol=0.0,
                chi_cap=10 ** 9, multiplets=False):
    """One time step dt of symmetric second-order two-site TDVP.

    Input: right-canonical MPS [C_1, B_2, ..., B_L] (centre on site 1).
    Left-to-right with tau = dt/2: for i = 1..L-1, Th = C_i B_{i+1};
    Th <- exp(-i tau H2_eff) Th; SVD Th = U S V^dag; A_i = U; C_{i+1} = S V^dag;
    update the left environment; if i < L-1, C_{i+1} <- exp(+i tau H1_eff) C_{i+1}.
    Then right-to-left, mirrored, with tau = dt/2, ending with the centre on
    site 1.  Returns the new MPS (same form) and the discarded weights."""
    L = len(mps)
    tau = dt / 2.0
    expm = (lambda f, v, z: lanczos_expm(f, v, z, tol=tol, maxdim=maxdim)[0])
    # right environments from the right-canonical tensors
    R = [None] * (L + 1)
    R[L] = empty_env()
    for k in range(L, 1, -1):
        R[k - 1] = right_env_update(R[k], mps[k - 1], k, t, U)
    Lf = [None] * (L + 1)
    Lf[0] = empty_env()
    mps = list(mps)
    disc = []
    C = mps[0]
    for i in range(1, L):
        Th = np.tensordot(C, mps[i], axes=([2], [0]))
        Th = expm(lambda x: heff2(Lf[i - 1], R[i + 1], x, i, t, U), Th, -1j * tau)
        a, s1, s2, b = Th.shape
        ops = left_row_ops(mps, i) if multiplets and not keep_all else None
        Um, S, Vh, d = _svd_split(Th.reshape(a * 4, 4 * b), keep_all, eps_tol, chi_cap, multiplets, ops)
        disc.append(d)
        mps[i - 1] = Um.reshape(a, 4, -1)
        C = (S[:, None] * Vh).reshape(-1, 4, b)
        Lf[i] = left_env_update(Lf[i - 1], mps[i - 1], i, t, U)
        if i < L - 1:
            C = expm(lambda x: heff1(Lf[i], R[i + 1], x, i + 1, t, U), C, +1j * tau)
    for i in range(L - 1, 0, -1):
        Th = np.tensordot(mps[i - 1], C, axes=([2], [0]))
        Th = expm(lambda x: heff2(Lf[i - 1], R[i + 1], x, i, t, U), Th, -1j * tau)
        a, s1, s2, b = Th.shape
        ops = left_row_ops(mps, i) if multiplets and not keep_all else None
        Um, S, Vh, d = _svd_split(Th.reshape(a * 4, 4 * b), keep_all, eps_tol, chi_cap, multiplets, ops)
        disc.append(d)
        mps[i] = Vh.reshape(-1, 4, b)
        C = (Um * S).reshape(a, 4, -1)
        R[i] = right_env_update(R[i + 1], mps[i], i + 1, t, U)
        if i > 1:
            C = expm(lambda x: heff1(Lf[i - 1], R[i], x, i, t, U), C, +1j * tau)
    mps[0] = C
    return mps, disc


def tdvp1_sweep(mps, dt, t, U, tol=1e-12, maxdim=40):
    """One time step dt of symmetric second-order one-site TDVP (supplementary
    section S2.2, projector splitting once the bond dimension is fixed).

    Input: right-canonical MPS [C_1, B_2, ..., B_L].  Left-to-right with
    tau = dt/2: for i = 1..L, C_i <- exp(-i tau H1_eff) C_i; for i < L,
    C_i = A_i R (QR), update the left environment, R <- exp(+i tau H0_eff) R
    with H0_eff = A_i^dag H1_eff A_i (the bond Hamiltonian between the new left
    environment and the right one), C_{i+1} = R B_{i+1}.  Then right-to-left,
    mirrored (C_i = R B_i by a QR of C_i^dag), ending with the centre on site 1."""
    L = len(mps)
    tau = dt / 2.0

    def expm(f, v, z):
        return lanczos_expm(f, v, z, tol=tol, maxdim=maxdim)[0]

    R = [None] * (L + 1)
    R[L] = empty_env()
    for k in range(L, 1, -1):
        R[k - 1] = right_env_update(R[k], mps[k - 1], k, t, U)
    Lf = [None] * (L + 1)
    Lf[0] = empty_env()
    mps = list(mps)
    for i in range(1, L + 1):
        C = expm(lambda v: heff1(Lf[i - 1], R[i], v, i, t, U), mps[i - 1], -1j * tau)
        if i == L:
            mps[i - 1] = C
            break
        a, _, b = C.shape
        Q, Rm = np.linalg.qr(C.reshape(a * 4, b))
        A = Q.reshape(a, 4, -1)
        mps[i - 1] = A
        Lf[i] = left_env_update(Lf[i - 1], A, i, t, U)

        def h0(x, A=A, i=i):
            y = heff1(Lf[i - 1], R[i], np.tensordot(A, x, axes=([2], [0])), i, t, U)
            return np.tensordot(A.conj(), y, axes=([0, 1], [0, 1]))
        x = expm(h0, Rm, +1j * tau)
        mps[i] = np.tensordot(x, mps[i], axes=([1], [0]))
    for i in range(L, 0, -1):
        C = expm(lambda v: heff1(Lf[i - 1], R[i], v, i, t, U), mps[i - 1], -1j * tau)
        if i == 1:
            mps[0] = C
            break
        a, _, b = C.shape
        Q, Rm = np.linalg.qr(C.reshape(a, 4 * b).conj().T)
        B = Q.conj().T.reshape(-1, 4, b)
        mps[i - 1] = B
        R[i - 1] = right_env_update(R[i], B, i, t, U)

        def h0(x, B=B, i=i):
            y = heff1(Lf[i - 1], R[i], np.tensordot(x, B, axes=([1], [0])), i, t, U)
            return np.tensordot(y, B.conj(), axes=([1, 2], [1, 2]))
        x = expm(h0, Rm.conj().T, +1j * tau)
        mps[i - 2] = np.tensordot(mps[i - 2], x, axes=([2], [0]))
    return mps
