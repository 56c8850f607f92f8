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


# ----------------------------------------------------------------------------
# Per-sector view of a two-site tensor and the multiplet truncation rule
# ----------------------------------------------------------------------------
def sector_matrices(blocks, left, right):
    """Reduced two-site tensor as one matrix per coupled sector x = (q_x, tj_x)
    of the bond being cut (the Wigner-Eckart grouping of supplementary section
    S2.1 applied to that bond): rows are the fusion partners (ia, s1) of x in
    ascending order, columns the partners (s2, ib), each a degeneracy block.
    Returns {x: (M_x, rows, cols)} with rows/cols lists of the partner keys."""
    fuse = lambda a, b: range(abs(a - b), a + b + 1, 2)
    out = {}
    for ia, (qa, tja, da) in enumerate(left):
        for s1, (q1, t1) in enumerate(MULTIPLETS):
            for tjx in fuse(tja, t1):
                out.setdefault((qa + q1, tjx), ([], []))[0].append((ia, s1))
    for (qx, tjx), (rows, cols) in out.items():
        for s2, (q2, t2) in enumerate(MULTIPLETS):
            for ib, (qb, tjb, db) in enumerate(right):
                if qx + q2 == qb and tjb in fuse(tjx, t2):
                    cols.append((s2, ib))
    res = {}
    for x, (rows, cols) in out.items():
        if not rows or not cols:
            continue
        ro = np.cumsum([0] + [left[r[0]][2] for r in rows])
        co = np.cumsum([0] + [right[c[1]][2] for c in cols])
        M = np.zeros((ro[-1], co[-1]), dtype=np.complex128)
        for i, (ia, s1) in enumerate(rows):
            for j, (s2, ib) in enumerate(cols):
                blk = blocks.get((ia, s1, x[1], s2, ib))
                if blk is not None:
                    M[ro[i]:ro[i + 1], co[j]:co[j + 1]] = blk
        res[x] = (M, rows, cols)
    return res


def sector_singular_values(blocks, left, right):
    """Reduced singular values of each coupled sector, descending:
    {(q_x, tj_x): array}.  The full-state singular values of the expanded
    tensor are these divided by sqrt(tj_x + 1), each tj_x + 1 times."""
    return {x: np.linalg.svd(M, compute_uv=False) for x, (M, _, _) in sector_matrices(blocks, left, right).items()}


def truncate_multiplets(svals, eps_tol, chi_cap):
    """The truncation of supplementary section S2.4 on whole multiplets.

    Every reduced singular value s of sector (q, tj) is one multiplet of
    tj + 1 full-state values s / sqrt(tj + 1) and full-state weight s^2.
    Multiplets are sorted by full-state value (descending; a value closer
    than 1e-9 of the largest one to its predecessor is a tie, and ties are
    ordered by q, then tj, ascending, then by position in the sector); the shortest prefix is kept
    whose discarded weight is at most eps_tol of the total, then cut before
    the first multiplet that would take the kept full-state dimension
    sum (tj + 1) above chi_cap; at least one multiplet stays.
    Returns ({(q, tj): kept count}, discarded weight / total weight)."""
    ents = []
    for (q, tj), s in svals.items():
        for idx, v in enumerate(s):
            ents.append((v / np.sqrt(tj + 1), q, tj, idx, v * v))
    ents.sort(key=lambda e: -e[0])
    # values closer than 1e-9 of the largest to their predecessor are ties
    tol = 1e-9 * (ents[0][0] if ents else 0.0)
    grouped, start = [], 0
    for i in range(1, len(ents) + 1):
        if i == len(ents) or ents[i - 1][0] - ents[i][0] > tol:
            grouped += sorted(ents[start:i], key=lambda e: (e[1], e[2], e[3]))
            start = i
    ents = grouped
    W = sum(e[4] for e in ents)
    keep, tail = len(ents), 0.0
    while keep > 1 and tail + ents[keep - 1][4] <= eps_tol * W:
        tail += ents[keep - 1][4]
        keep -= 1
    chi, p = 0, 0
    while p < keep and (p == 0 or chi + ents[p][2] + 1 <= chi_cap):
        chi += ents[p][2] + 1
        p += 1
    kept = {x: 0 for x in svals}
    for e in ents[:p]:
        kept[(e[1], e[2])] += 1
    kw = sum(e[4] for e in ents[:p])
    return kept, ((W - kw) / W if W > 0 else 0.0)


def _spin_matrices(tj):
    """(J+, Jz) of spin tj/2 in the basis of descending m (Condon-Shortley)."""
    n = tj + 1
    ms = [(tj - 2 * i) / 2.0 for i in range(n)]
    jp = np.zeros((n, n))
    j = tj / 2.0
    for i in range(1, n):      # J+ |m> = sqrt((j - m)(j + m + 1)) |m + 1>, m = ms[i], m + 1 = ms[i - 1]
        m = ms[i]
        jp[i - 1, i] = np.sqrt((j - m) * (j + m + 1))
    return jp, np.diag(ms)


def row_quantum_ops(left, k):
    """(2 S^z, T^2) of the block made of everything left of the bond `left`
    plus site k, on the row space (full left index, Jordan-Wigner state of
    site k) of a two-site tensor reshaped to [chi_left * 4, 4 * chi_right].
    The bond part acts on the magnetic index of every sector multiplet
    (descending m); the site part is the eta pseudospin of site k,
    T+ = (-1)^k c+_up c+_dn, and S^z = (n_up - n_dn) / 2."""
    from .fermions import A_UP, A_DN
    _, dim = bond_offsets(left)
    Jp = np.zeros((dim, dim))
    Jz = np.zeros((dim, dim))
    Q = np.zeros(dim)
    o = 0
    for (q, tj, d) in left:
        jp, jz = _spin_matrices(tj)
        for _ in range(d):
            Jp[o:o + tj + 1, o:o + tj + 1] = jp
            Jz[o:o + tj + 1, o:o + tj + 1] = jz
            Q[o:o + tj + 1] = q
            o += tj + 1
    tp = (-1.0) ** k * (A_UP.T @ A_DN.T)
    nu, nd = A_UP.T @ A_UP, A_DN.T @ A_DN
    tz = 0.5 * (nu + nd - np.eye(4))
    I4, Id = np.eye(4), np.eye(dim)
    Tp = np.kron(Jp, I4) + np.kron(Id, tp)
    Tz = np.kron(Jz, I4) + np.kron(Id, tz)
    T2 = Tp @ Tp.T + Tz @ Tz - Tz
    Sz2 = np.kron(np.diag(Q), I4) + np.kron(Id, nu - nd)
    return Sz2, T2
