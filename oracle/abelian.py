"""Expansion of U(1)_N x U(1)_Sz block tensors to full tensors.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's comparison runs use only the two abelian symmetries (particle
number and S^z; Table 1, Table S1).  With them every bond sector is one
(N, 2 S^z) label of everything left of the bond and every local state is its
own sector, so a block tensor is just the full tensor cut into sector pairs;
the written convention shared with the library is only the labelling:

* bond sector ``(sz2, N, d)``: 2 S^z, particle number, degeneracy;
* full index of a bond: sectors in list order, degeneracy index inside;
* local state s = n_up + 2 n_dn (the basis of ``oracle.fermions``), carrying
  N = n_up + n_dn and 2 S^z = n_up - n_dn;
* site tensors, key (a, s, b), block d_a x d_b = M_full[a-range, s, b-range];
* two-site tensors, key (a, s1, s2, b);
* environments, key (out, w, in): w = 0 the block Hamiltonian, w = 1..4 the
  single components of the doublet channels of ``oracle.dense`` (w = 1, 2:
  channel 'D+' components kappa = +1/2, -1/2; w = 3, 4: 'D-'), i.e.
  E_w block = E_dense[channel][out-range, kappa, in-range].
"""
import numpy as np

LOCAL_N = [0, 1, 1, 2]
LOCAL_SZ2 = [0, 1, -1, 0]
# dense channel and component of the abelian channel w = 1..4
CHANNEL = {1: (1, 0), 2: (1, 1), 3: (2, 0), 4: (2, 1)}


def offsets(bond):
    """Start of each sector in the full bond index, and the full dimension."""
    off = np.cumsum([0] + [d for _, _, d in bond])
    return off[:-1], int(off[-1])


def expand_site(blocks, left, right):
    """{(a, s, b): d_a x d_b} -> full M[chi_l, 4, chi_r]."""
    lo, ln = offsets(left)
    ro, rn = offsets(right)
    M = np.zeros((ln, 4, rn), complex)
    for (a, s, b), blk in blocks.items():
        M[lo[a]:lo[a] + left[a][2], s, ro[b]:ro[b] + right[b][2]] = blk
    return M


def expand_theta(blocks, left, right):
    """{(a, s1, s2, b): d_a x d_b} -> full Th[chi_l, 4, 4, chi_r]."""
    lo, ln = offsets(left)
    ro, rn = offsets(right)
    Th = np.zeros((ln, 4, 4, rn), complex)
    for (a, s1, s2, b), blk in blocks.items():
        Th[lo[a]:lo[a] + left[a][2], s1, s2, ro[b]:ro[b] + right[b][2]] = blk
    return Th


def expand_env(blocks, bond):
    """{(out, w, in): d_out x d_in} -> the dense environment {0: E[chi, 1, chi],
    1: E[chi, 2, chi], 2: E[chi, 2, chi]} of ``oracle.dense``."""
    o, n = offsets(bond)
    env = {0: np.zeros((n, 1, n), complex), 1: np.zeros((n, 2, n), complex), 2: np.zeros((n, 2, n), complex)}
    for (io, w, ii), blk in blocks.items():
        ch, kap = (0, 0) if w == 0 else CHANNEL[w]
        env[ch][o[io]:o[io] + bond[io][2], kap, o[ii]:o[ii] + bond[ii][2]] = blk
    return env


def restrict_env(env, bond, keys):
    """Inverse of expand_env on the listed keys: the sector blocks of a dense
    environment."""
    o, _ = offsets(bond)
    out = {}
    for io, w, ii in keys:
        ch, kap = (0, 0) if w == 0 else CHANNEL[w]
        out[(io, w, ii)] = env[ch][o[io]:o[io] + bond[io][2], kap, o[ii]:o[ii] + bond[ii][2]]
    return out


def restrict_theta(Th, left, right, keys):
    lo, _ = offsets(left)
    ro, _ = offsets(right)
    return {(a, s1, s2, b): Th[lo[a]:lo[a] + left[a][2], s1, s2, ro[b]:ro[b] + right[b][2]]
            for a, s1, s2, b in keys}


def restrict_site(M, left, right, keys):
    lo, _ = offsets(left)
    ro, _ = offsets(right)
    return {(a, s, b): M[lo[a]:lo[a] + left[a][2], s, ro[b]:ro[b] + right[b][2]] for a, s, b in keys}
