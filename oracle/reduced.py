"""Expansion of U(1)_spin x SU(2)_charge reduced tensors to full tensors.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper decomposes every bond space into degeneracy spaces times pseudospin
multiplets (supplementary section S2.1, equation for the bond-space
decomposition; the Wigner-Eckart grouping of the main text).  It does not fix
a normalisation or a fusion tree, so the library and this oracle share the
following written convention (and nothing else):

Labels
  Bond sector ``(q, tj)``: q = 2 S^z of everything left of the bond, tj = 2 T
  (pseudospin of everything left of the bond); degeneracy ``d``.
  Local multiplets of site k (1-based):
     s = 0: (q= 0, tj=1)  components m=+1/2 -> |up dn>,  m=-1/2 -> (-1)^k |0>
     s = 1: (q=+1, tj=0)  |up>
     s = 2: (q=-1, tj=0)  |dn>
  (the staggered phase makes the pair a standard doublet of the
  eta-pairing pseudospin T+ = sum_k (-1)^k c+_k,up c+_k,dn).

Full index of a bond: sectors in list order; inside a sector, degeneracy index
slow and magnetic component fast, components in descending m.

Tensors (C(..) is the Condon-Shortley Clebsch-Gordan coefficient):
  A  (left-canonical site tensor, block key (a, s, b), d_a x d_b):
       A_full[(a,al,ma),(s,mu),(b,be,mb)] = A[al,be] C(ja ma; js mu | jb mb)
  B  (right-canonical site tensor, same key):
       B_full = B[al,be] C(ja ma; js mu | jb mb) sqrt((2ja+1)/(2jb+1))
  C1 (one-site centre tensor, same key):
       C_full = C[al,be] C(ja ma; js mu | jb mb) / sqrt(2jb+1)
  Theta (two-site tensor, key (a, s1, tjx, s2, b), d_a x d_b), tree
       ((a x s1) -> x) x s2 -> b:
       Th_full = Th[al,be] sum_mx C(ja ma; js1 mu1 | jx mx) C(jx mx; js2 mu2 | jb mb) / sqrt(2jb+1)
  With these, the flat Frobenius norm of the reduced blocks equals the norm of
  the state when everything left of the centre is left-canonical and
  everything right of it right-canonical.

Environments (block key (out, w, in), stored d_out x d_in):
  channel w = 0 'H' (tj_w=0, q_w=0), 1 'D+' (tj_w=1, q_w=+1), 2 'D-' (tj_w=1, q_w=-1)
       E_full[(out,al',m'), kappa, (in,al,m)] = E[al',al] C(j_in m; j_w kappa | j_out m')
  Left environments hold <Phi_out| O |Phi_in> over the left block basis, right
  environments <Psi_out| Q |Psi_in> over the right block basis, with the
  operators listed in ``dense.left_channel_ops`` / ``dense.right_channel_ops``.
"""
import numpy as np

from .cg import cg_tensor

MULTIPLETS = [(0, 1), (1, 0), (-1, 0)]       # (q, tj) of s = 0, 1, 2
CHANNELS = [(0, 0), (1, 1), (-1, 1)]         # (q_w, tj_w) of w = 0 'H', 1 'D+', 2 'D-'


def local_basis(k):
    """4x4 matrix from multiplet components (s=0 m=+1/2, s=0 m=-1/2, s=1, s=2)
    to the Jordan-Wigner local basis [|0>,|up>,|dn>,|up dn>] of site k."""
    U = np.zeros((4, 4))
    U[3, 0] = 1.0
    U[0, 1] = (-1.0) ** k
    U[1, 2] = 1.0
    U[2, 3] = 1.0
    return U


_COMP0 = [0, 2, 3]   # first multiplet-component column of s = 0, 1, 2


def bond_offsets(bond):
    """Full-index offset of each sector of a bond [(q, tj, d), ...] and the
    total full dimension."""
    offs = []
    o = 0
    for (q, tj, d) in bond:
        offs.append(o)
        o += d * (tj + 1)
    return offs, o


def full_dim(bond):
    return bond_offsets(bond)[1]


def expand_site(kind, blocks, left, right, k):
    """Full tensor [chi_left, 4, chi_right] of a one-site reduced tensor.

    kind: 'A', 'B' or 'C'; blocks: {(ia, s, ib): (d_a x d_b) array};
    left/right: bonds [(q, tj, d)]; k: 1-based site index."""
    lo, ldim = bond_offsets(left)
    ro, rdim = bond_offsets(right)
    U = local_basis(k)
    out = np.zeros((ldim, 4, rdim), dtype=np.complex128)
    for (ia, s, ib), blk in blocks.items():
        qa, tja, da = left[ia]
        qb, tjb, db = right[ib]
        qs, tjs = MULTIPLETS[s]
        assert qb == qa + qs, "block violates U(1) fusion"
        cg = cg_tensor(tja, tjs, tjb)                     # [ma, mu, mb]
        if kind == "A":
            f = 1.0
        elif kind == "B":
            f = np.sqrt((tja + 1) / (tjb + 1))
        elif kind == "C":
            f = 1.0 / np.sqrt(tjb + 1)
        else:
            raise ValueError(kind)
        Us = U[:, _COMP0[s]:_COMP0[s] + tjs + 1]           # [jw, mu]
        mt = f * np.einsum("amb,jm->ajb", cg, Us)           # [ma, jw, mb]
        full = np.einsum("xy,ajb->xajyb", np.asarray(blk), mt)
        full = full.reshape(da * (tja + 1), 4, db * (tjb + 1))
        out[lo[ia]:lo[ia] + da * (tja + 1), :, ro[ib]:ro[ib] + db * (tjb + 1)] += full
    return out


def expand_theta(blocks, left, right, i):
    """Full two-site tensor [chi_left, 4, 4, chi_right] for sites (i, i+1).
    blocks: {(ia, s1, tjx, s2, ib): (d_a x d_b) array}."""
    lo, ldim = bond_offsets(left)
    ro, rdim = bond_offsets(right)
    U1 = local_basis(i)
    U2 = local_basis(i + 1)
    out = np.zeros((ldim, 4, 4, rdim), dtype=np.complex128)
    for (ia, s1, tjx, s2, ib), blk in blocks.items():
        qa, tja, da = left[ia]
        qb, tjb, db = right[ib]
        q1, tj1 = MULTIPLETS[s1]
        q2, tj2 = MULTIPLETS[s2]
        assert qb == qa + q1 + q2, "block violates U(1) fusion"
        c1 = cg_tensor(tja, tj1, tjx)                      # [ma, mu1, mx]
        c2 = cg_tensor(tjx, tj2, tjb)                      # [mx, mu2, mb]
        tree = np.einsum("amx,xnb->amnb", c1, c2) / np.sqrt(tjb + 1)
        u1 = U1[:, _COMP0[s1]:_COMP0[s1] + tj1 + 1]
        u2 = U2[:, _COMP0[s2]:_COMP0[s2] + tj2 + 1]
        mt = np.einsum("amnb,jm,kn->ajkb", tree, u1, u2)
        full = np.einsum("xy,ajkb->xajkyb", np.asarray(blk), mt)
        full = full.reshape(da * (tja + 1), 4, 4, db * (tjb + 1))
        out[lo[ia]:lo[ia] + da * (tja + 1), :, :, ro[ib]:ro[ib] + db * (tjb + 1)] += full
    return out


def expand_env(blocks, bond):
    """Full environment, one array per channel: {w: [chi, n_kappa, chi]}
    with n_kappa = 1 for 'H' and 2 for 'D+'/'D-' (kappa = +1/2, -1/2).
    blocks: {(iout, w, iin): (d_out x d_in) array}."""
    offs, dim = bond_offsets(bond)
    out = {w: np.zeros((dim, CHANNELS[w][1] + 1, dim), dtype=np.complex128) for w in range(3)}
    for (io, w, ii), blk in blocks.items():
        qo, tjo, do = bond[io]
        qi, tji, di = bond[ii]
        qw, tjw = CHANNELS[w]
        assert qo == qi + qw, "env block violates U(1) selection rule"
        cg = cg_tensor(tji, tjw, tjo)                     # [m, kappa, m']
        mt = np.transpose(cg, (2, 1, 0))                   # [m', kappa, m]
        full = np.einsum("xy,akb->xakyb", np.asarray(blk), mt)
        full = full.reshape(do * (tjo + 1), tjw + 1, di * (tji + 1))
        out[w][offs[io]:offs[io] + do * (tjo + 1), :, offs[ii]:offs[ii] + di * (tji + 1)] += full
    return out
