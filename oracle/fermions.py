"""Jordan-Wigner fermions, the 1D Fermi-Hubbard Hamiltonian and exact evolution.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (the reading of the paper used throughout the oracle):

* Sites are numbered 1..L (the paper's Eq. (2) puts spin up on site 1).
* The 2L fermion modes are ordered (1 up, 1 down, 2 up, 2 down, ...).
* The local basis of one site is indexed by ``n_up + 2 n_dn``:
  0 = |0>, 1 = |up>, 2 = |dn>, 3 = |up dn> = c+_up c+_dn |0>.
* A full state vector is ``psi[s_1, s_2, ..., s_L]`` flattened in C order
  (site 1 slowest); basis state |s_1 ... s_L> is the mode-ordered product of
  creation operators acting on the vacuum.
* ``hubbard(L, t, U)`` is the paper's Eq. (1) on an open chain,
  H = -t sum_<ij>,s (c+_is c_js + h.c.) + U sum_i n_i,up n_i,dn.
  ``symmetric=True`` replaces the interaction by U (n_up - 1/2)(n_dn - 1/2),
  the particle-hole symmetric form that commutes with the eta-pairing
  pseudospin of supplementary section S2.1 (Eq. (1)'s own form does not:
  [H, T+] = U T+).  At half filling the two differ by the constant U L / 4.
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import expm_multiply

# ---- one-site operators in the local basis [|0>, |up>, |dn>, |up dn>] -------
# a_up annihilates the up fermion (first mode of the site, no string).
A_UP = np.zeros((4, 4))
A_UP[0, 1] = 1.0          # a_up |up>    = |0>
A_UP[2, 3] = 1.0          # a_up |up dn> = a_up c+_up c+_dn |0> = |dn>
# a_dn carries the on-site string (-1)^{n_up} (second mode of the site).
A_DN = np.zeros((4, 4))
A_DN[0, 2] = 1.0          # a_dn |dn>    = |0>
A_DN[1, 3] = -1.0         # a_dn c+_up c+_dn |0> = -c+_up a_dn c+_dn |0> = -|up>
PARITY = np.diag([1.0, -1.0, -1.0, 1.0])
N_UP = A_UP.T @ A_UP
N_DN = A_DN.T @ A_DN
EYE4 = np.eye(4)


def site_op(op, i, L):
    """Operator ``op`` on site i (1-based) of an L-site chain, no string."""
    return sp.kron(sp.kron(sp.identity(4 ** (i - 1), format="csr"), sp.csr_matrix(op)),
                   sp.identity(4 ** (L - i), format="csr"), format="csr")


def annihilator(i, spin, L):
    """c_{i,spin} (spin 0 = up, 1 = down) with its Jordan-Wigner string."""
    string = sp.identity(1, format="csr")
    for _ in range(i - 1):
        string = sp.kron(string, sp.csr_matrix(PARITY), format="csr")
    local = A_UP if spin == 0 else A_DN
    return sp.kron(sp.kron(string, sp.csr_matrix(local)), sp.identity(4 ** (L - i), format="csr"),
                   format="csr")


def hubbard(L, t=1.0, U=4.0, symmetric=False):
    """Sparse Hamiltonian of Eq. (1) on an open chain of L sites."""
    dim = 4 ** L
    H = sp.csr_matrix((dim, dim), dtype=np.float64)
    c = {(i, s): annihilator(i, s, L) for i in range(1, L + 1) for s in (0, 1)}
    for i in range(1, L):
        for s in (0, 1):
            hop = c[(i, s)].T @ c[(i + 1, s)]
            H = H - t * (hop + hop.T)
    for i in range(1, L + 1):
        nu = c[(i, 0)].T @ c[(i, 0)]
        nd = c[(i, 1)].T @ c[(i, 1)]
        if symmetric:
            eye = sp.identity(dim, format="csr")
            H = H + U * ((nu - 0.5 * eye) @ (nd - 0.5 * eye))
        else:
            H = H + U * (nu @ nd)
    return H.tocsr()


def pseudospin(L):
    """(T+, T-, Tz) of supplementary section S2.1: T+ = sum_i (-1)^i c+_i,up c+_i,dn,
    Tz = (N - L)/2."""
    c = {(i, s): annihilator(i, s, L) for i in range(1, L + 1) for s in (0, 1)}
    dim = 4 ** L
    Tp = sp.csr_matrix((dim, dim))
    N = sp.csr_matrix((dim, dim))
    for i in range(1, L + 1):
        Tp = Tp + (-1) ** i * (c[(i, 0)].T @ c[(i, 1)].T)
        N = N + c[(i, 0)].T @ c[(i, 0)] + c[(i, 1)].T @ c[(i, 1)]
    Tz = 0.5 * (N - L * sp.identity(dim))
    return Tp.tocsr(), Tp.T.tocsr(), Tz.tocsr()


def neel_state(L):
    """The Neel product state of Eq. (2): up on odd sites, down on even sites,
    as the basis state |up dn up dn ...> of the Jordan-Wigner tensor product
    (Eq. (2)'s ordering of the creation operators changes only a global sign)."""
    psi = np.zeros(4 ** L, dtype=np.complex128)
    idx = 0
    for i in range(1, L + 1):
        idx = idx * 4 + (1 if i % 2 == 1 else 2)
    psi[idx] = 1.0
    return psi


def local_expectations(psi, L):
    """<n_i,up>, <n_i,dn>, <n_i,up n_i,dn> for i = 1..L (arrays of length L)."""
    p = np.abs(np.asarray(psi).reshape([4] * L)) ** 2
    nu = np.empty(L)
    nd = np.empty(L)
    dd = np.empty(L)
    for i in range(L):
        marg = p.sum(axis=tuple(k for k in range(L) if k != i))
        nu[i] = marg[1] + marg[3]
        nd[i] = marg[2] + marg[3]
        dd[i] = marg[3]
    return nu, nd, dd


def evolve(H, psi0, times):
    """Exact psi(t) = exp(-i H t) psi0 for each t in ``times`` (ascending,
    equally spaced from 0).  Returns an array of shape (len(times), dim)."""
    times = np.asarray(times, dtype=float)
    if len(times) == 1:
        return expm_multiply(-1j * times[0] * H, psi0)[None, :]
    return expm_multiply(-1j * H, psi0, start=times[0], stop=times[-1], num=len(times),
                         endpoint=True)


def free_fermion_density(L, t_h, times, n0):
    """Closed form at U = 0 for a state whose one-body density matrix is
    diagonal (a Fock state such as the Neel state): the occupation of each
    spin species evolves as n_i(t) = sum_j |[exp(-i h t)]_ij|^2 n_j(0), with h
    the open-chain single-particle hopping matrix."""
    h = np.zeros((L, L))
    for i in range(L - 1):
        h[i, i + 1] = h[i + 1, i] = -t_h
    w, v = np.linalg.eigh(h)
    out = []
    for tt in times:
        u = (v * np.exp(-1j * w * tt)) @ v.T
        out.append((np.abs(u) ** 2) @ n0)
    return np.array(out)
