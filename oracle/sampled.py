"""Sector-restricted evaluation of single output blocks.

TEST INFRASTRUCTURE ONLY (see the package docstring).

At the paper's bond dimensions the full expanded problem does not fit in
memory, but one output block of the effective Hamiltonian only receives
contributions from input blocks whose left sector is the output's left
sector or one connected to it by a left-environment block, and whose right
sector is likewise connected on the right.  Restricting both bonds to those
sectors and applying the dense definition (``dense.heff2``) to the
restricted, expanded tensors gives that output block exactly; nothing else
is approximated.  ``heff2_block_cross`` reaches the same block through three
smaller restricted problems (inclusion-exclusion over the terms), for blocks
whose fully connected restriction is too large to expand.
"""
import numpy as np

from . import dense as D
from . import reduced as R


def _restrict(bond, keep):
    keep = sorted(set(keep))
    sub = [bond[i] for i in keep]
    remap = {old: new for new, old in enumerate(keep)}
    return sub, remap


def _eval_restricted(left, right, Lenv, Renv, theta, out_key, site, t, U, lk, rk):
    """The dense definition on the bonds restricted to the sectors lk (left)
    and rk (right), projected on the reduced output block out_key."""
    ia, s1, tjx, s2, ib = out_key
    lsub, lmap = _restrict(left, lk)
    rsub, rmap = _restrict(right, rk)
    Ls = {(lmap[a], w, lmap[b]): v for (a, w, b), v in Lenv.items() if a in lmap and b in lmap}
    Rs = {(rmap[a], w, rmap[b]): v for (a, w, b), v in Renv.items() if a in rmap and b in rmap}
    Ts = {(lmap[k[0]], k[1], k[2], k[3], rmap[k[4]]): v for k, v in theta.items()
          if k[0] in lmap and k[4] in rmap}
    out = D.heff2(R.expand_env(Ls, lsub), R.expand_env(Rs, rsub), R.expand_theta(Ts, lsub, rsub, site), site, t, U)
    da, db = left[ia][2], right[ib][2]
    lo, _ = R.bond_offsets(lsub)
    ro, _ = R.bond_offsets(rsub)
    tja, tjb = left[ia][1], right[ib][1]
    unit = R.expand_theta({(0, s1, tjx, s2, 0): np.ones((1, 1))}, [(left[ia][0], tja, 1)],
                          [(right[ib][0], tjb, 1)], site)
    a0, b0 = lo[lmap[ia]], ro[rmap[ib]]
    sl = out[a0:a0 + da * (tja + 1), :, :, b0:b0 + db * (tjb + 1)].reshape(da, tja + 1, 4, 4, db, tjb + 1)
    return np.einsum("xajkyb,ajkb->xy", sl, unit.reshape(tja + 1, 4, 4, tjb + 1))


def heff2_block_cross(left, right, Lenv, Renv, theta, out_key, site, t, U):
    """The same output block by inclusion-exclusion over three smaller
    restricted problems.  Every term of the effective Hamiltonian acts on the
    left block only (keeping the right sector), on the right block only
    (keeping the left sector), or on the two sites only.  So the block is
      P(left connected, {ib}) + P({ia}, right connected) - P({ia}, {ib}),
    P(lk, rk) being the dense definition on bonds restricted to lk and rk:
    the first holds every left term, the second every right term, each also
    the local terms and the diagonal block-Hamiltonian term of the other side
    (the only term a single sector keeps there), which the third removes once."""
    ia, ib = out_key[0], out_key[4]
    lconn = [ia] + [k[2] for k in Lenv if k[0] == ia]
    rconn = [ib] + [k[2] for k in Renv if k[0] == ib]
    args = (left, right, Lenv, Renv, theta, out_key, site, t, U)
    return (_eval_restricted(*args, lconn, [ib]) + _eval_restricted(*args, [ia], rconn)
            - _eval_restricted(*args, [ia], [ib]))


def heff2_block(left, right, Lenv, Renv, theta, out_key, site, t, U):
    """Output block ``out_key = (ia, s1, tjx, s2, ib)`` of the two-site
    effective Hamiltonian applied to ``theta``.

    left/right: bonds [(q, tj, d)]; Lenv/Renv: {(iout, w, iin): block};
    theta: {(ia, s1, tjx, s2, ib): block}.  Returns the reduced block
    (d_a x d_b) and the restricted full dimensions used."""
    ia, s1, tjx, s2, ib = out_key
    lk = [ia] + [k[2] for k in Lenv if k[0] == ia]
    rk = [ib] + [k[2] for k in Renv if k[0] == ib]
    lsub, lmap = _restrict(left, lk)
    rsub, rmap = _restrict(right, rk)
    Ls = {(lmap[a], w, lmap[b]): v for (a, w, b), v in Lenv.items() if a in lmap and b in lmap}
    Rs = {(rmap[a], w, rmap[b]): v for (a, w, b), v in Renv.items() if a in rmap and b in rmap}
    Ts = {(lmap[k[0]], k[1], k[2], k[3], rmap[k[4]]): v for k, v in theta.items()
          if k[0] in lmap and k[4] in rmap}
    Lf = R.expand_env(Ls, lsub)
    Rf = R.expand_env(Rs, rsub)
    Th = R.expand_theta(Ts, lsub, rsub, site)
    out = D.heff2(Lf, Rf, Th, site, t, U)
    # project the output onto the reduced block: the fusion trees are orthonormal,
    # so the reduced element is the overlap with the expanded unit block
    key = (lmap[ia], s1, tjx, s2, rmap[ib])
    da, db = left[ia][2], right[ib][2]
    lo, _ = R.bond_offsets(lsub)
    ro, _ = R.bond_offsets(rsub)
    tja, tjb = left[ia][1], right[ib][1]
    unit = R.expand_theta({(0, s1, tjx, s2, 0): np.ones((1, 1))}, [(left[ia][0], tja, 1)],
                          [(right[ib][0], tjb, 1)], site)
    sl = out[lo[key[0]]:lo[key[0]] + da * (tja + 1), :, :, ro[key[4]]:ro[key[4]] + db * (tjb + 1)]
    sl = sl.reshape(da, tja + 1, 4, 4, db, tjb + 1)
    red = np.einsum("xajkyb,ajkb->xy", sl, unit.reshape(tja + 1, 4, 4, tjb + 1))
    return red, (Th.shape[0], Th.shape[3])


def restricted_dims(left, right, Lenv_keys, Renv_keys, out_key):
    """Full dimensions of the restricted problem for an output block (used to
    pick samples that finish quickly)."""
    ia, ib = out_key[0], out_key[4]
    lk = {ia} | {k[2] for k in Lenv_keys if k[0] == ia}
    rk = {ib} | {k[2] for k in Renv_keys if k[0] == ib}
    return (sum(left[i][2] * (left[i][1] + 1) for i in lk), sum(right[i][2] * (right[i][1] + 1) for i in rk))
