"""Seeded synthetic inputs shaped like the paper's L=60 Neel-quench states.

This module only draws random numbers and lays out shapes.  It holds none
of the method's arithmetic (no coupling coefficients, no Hamiltonian, no
contraction); the library and the oracle both consume what it returns.

Shapes follow the paper's Table S2 (32 sectors at the middle bond of the
chi ~ 30 000 run): sector degeneracies d_(q,j) are a Gaussian in the U(1)
label q and the SU(2) label j, fitted to that table, with a seeded +-10 %
log-normal jitter and largest-remainder rounding so that the full-state bond
dimension sum_d d (2j+1) hits the requested chi exactly.

Labels: a bond sector is (q, tj) with q = 2 S^z and tj = 2T of the block left
of the bond.  For a left block of l sites q and tj have the parity of l
(q - tj = l mod 2).  The three local multiplets of a Hubbard site are
(q, tj) = (0, 1), (+1, 0), (-1, 0).
"""
import numpy as np

LOCAL = [(0, 1), (1, 0), (-1, 0)]
TABLE_S2_FIT = (-0.69, 1.69, 0.60, 0.72)      # (mu_q, sigma_q, mu_j, sigma_j)


def _rng(seed, *key):
    return np.random.default_rng([int(seed) & 0x7FFFFFFF] + [int(k) + 4096 for k in key])


def sector_profile(chi, seed, parity=0, shape=TABLE_S2_FIT, jitter=0.10, qmax=8, tjmax=8):
    """Sectors [(q, tj, d)] sorted by (q, tj) with sum d (tj+1) == chi.

    parity: l mod 2 of the left block (q - tj = parity mod 2)."""
    mu_q, sg_q, mu_j, sg_j = shape
    rng = _rng(seed, 1, chi, parity)
    labels = [(q, tj) for q in range(-qmax, qmax + 1) for tj in range(0, tjmax + 1)
              if (q - tj - parity) % 2 == 0]
    w = np.array([np.exp(-(q - mu_q) ** 2 / (2 * sg_q ** 2) - (tj / 2 - mu_j) ** 2 / (2 * sg_j ** 2))
                  for q, tj in labels])
    w *= np.exp(jitter * rng.standard_normal(len(labels)))
    mult = np.array([tj + 1 for _, tj in labels])
    target = w * chi / np.sum(w * mult)
    d = np.floor(target).astype(np.int64)
    rem = chi - int(np.sum(d * mult))
    order = np.argsort(-(target - d), kind="stable")
    while rem > 0:
        placed = False
        for i in order:
            if mult[i] <= rem:
                d[i] += 1
                rem -= mult[i]
                placed = True
                if rem == 0:
                    break
        if not placed:
            raise ValueError("cannot round the profile to chi exactly")
    return [(q, tj, int(di)) for (q, tj), di in zip(labels, d) if di > 0]


def lognormal_profile(chi, seed, parity=0, median=200.0, sigma=1.0, lo=8, hi=2048, qmax=8, tjmax=8):
    """Sectors [(q, tj, d)] over the label window (q in [-qmax, qmax],
    2j in [0, tjmax], q - tj = parity mod 2) with degeneracies drawn from a
    log-normal (median, sigma), clipped to [lo, hi], then rescaled and rounded
    (largest remainder) so that sum d (tj+1) == chi."""
    rng = _rng(seed, 3, chi, parity)
    labels = [(q, tj) for q in range(-qmax, qmax + 1) for tj in range(0, tjmax + 1)
              if (q - tj - parity) % 2 == 0]
    raw = np.clip(np.exp(np.log(median) + sigma * rng.standard_normal(len(labels))), lo, hi)
    mult = np.array([tj + 1 for _, tj in labels])
    target = raw * chi / np.sum(raw * mult)
    d = np.floor(target).astype(np.int64)
    rem = chi - int(np.sum(d * mult))
    order = np.argsort(-(target - d), kind="stable")
    while rem > 0:
        placed = False
        for i in order:
            if mult[i] <= rem:
                d[i] += 1
                rem -= mult[i]
                placed = True
                if rem == 0:
                    break
        if not placed:
            raise ValueError("cannot round the profile to chi exactly")
    return [(q, tj, int(di)) for (q, tj), di in zip(labels, d) if di > 0]


def chi_full(bond):
    return sum(d * (tj + 1) for _, tj, d in bond)


def chi_su2(bond):
    return sum(d for _, _, d in bond)


def _fuse(tja, tjs):
    return range(abs(tja - tjs), tja + tjs + 1, 2)


def _max_mult(n):
    """Largest multiplicity of every (q, tj) in a block of n sites, by the
    multiplet counting recursion (pure integer bookkeeping)."""
    cur = {(0, 0): 1}
    for _ in range(n):
        nxt = {}
        for (q, tj), m in cur.items():
            for qs, tjs in LOCAL:
                for tjb in _fuse(tj, tjs):
                    nxt[(q + qs, tjb)] = nxt.get((q + qs, tjb), 0) + m
        cur = nxt
    return cur


def complex_normal(shape, seed, *key):
    r = _rng(seed, 2, *key)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def block_data(keys, dims, seed, tag=0):
    """Independent complex-normal blocks keyed by their labels, so that the
    values do not depend on the order in which blocks are listed."""
    return {tuple(k): complex_normal(tuple(dm), seed, tag, *k) for k, dm in zip(keys, dims)}


def random_bonds(L, chi, seed, center=1, profile_seed=None):
    """The bonds [(q, tj, d)] of ``random_mps`` (same arguments) without its
    site tensors."""
    return random_mps(L, chi, seed, center, profile_seed, bonds_only=True)


def random_mps(L, chi, seed, center=1, profile_seed=None, bonds_only=False):
    """Random MPS of L sites in mixed-canonical form with the centre on
    ``center``: sites left of it left-canonical, right of it right-canonical.

    Each bond k (k sites to its left) gets the Table-S2-shaped profile at
    full-state dimension ``chi`` (parity k mod 2), capped sector by sector by
    what the sites on both sides can hold and by the isometry condition of
    the neighbouring tensor, so the tensors exist.

    Returns (bonds, sites): bonds[k] = [(q, tj, d)] for k = 0..L;
    sites[k-1] = {(ia, s, ib): d_a x d_b complex array} for site k, in the
    block conventions of the library (A left-canonical: sum A^dag A = 1 per
    output sector; B right-canonical: sum B B^dag = 1 per input sector; the
    centre normalised to unit Frobenius norm)."""
    ps = seed if profile_seed is None else profile_seed
    left_cap = [_max_mult(k) for k in range(L + 1)]
    bonds = [None] * (L + 1)
    bonds[0] = [(0, 0, 1)]
    bonds[L] = [(0, 0, 1)]
    for k in range(1, L):
        prof = {(q, tj): d for q, tj, d in sector_profile(chi, ps + 7919 * k, parity=k % 2)}
        capl = left_cap[k]
        capr = left_cap[L - k]
        bond = []
        for (q, tj), d in prof.items():
            c = min(d, capl.get((q, tj), 0), capr.get((-q, tj), 0))
            if c > 0:
                bond.append((q, tj, c))
        # sectors that the tiny edges need even if the profile misses them
        for (q, tj), m in capl.items():
            if (q, tj) not in prof and capr.get((-q, tj), 0) > 0 and chi_full(bond) < chi and m > 0 \
                    and min(k, L - k) <= 3:
                bond.append((q, tj, min(m, capr[(-q, tj)])))
        bonds[k] = sorted(bond)
    # enforce isometry feasibility: left part grows from the left, right part from the right
    for k in range(1, center):
        prev = bonds[k - 1]
        nb = []
        for q, tj, d in bonds[k]:
            rows = sum(da for (qa, tja, da) in prev for qs, tjs in LOCAL
                       if qa + qs == q and tj in _fuse(tja, tjs))
            if min(d, rows) > 0:
                nb.append((q, tj, min(d, rows)))
        bonds[k] = nb
    for k in range(L - 1, center - 1, -1):
        nxt = bonds[k + 1]
        nb = []
        for q, tj, d in bonds[k]:
            cols = sum(db for (qb, tjb, db) in nxt for qs, tjs in LOCAL
                       if q + qs == qb and tjb in _fuse(tj, tjs))
            if min(d, cols) > 0:
                nb.append((q, tj, min(d, cols)))
        bonds[k] = nb
    if bonds_only:
        return bonds
    sites = [None] * L
    for k in range(1, L + 1):
        lb, rb = bonds[k - 1], bonds[k]
        keys, dims = [], []
        for ia, (qa, tja, da) in enumerate(lb):
            for s, (qs, tjs) in enumerate(LOCAL):
                for ib, (qb, tjb, db) in enumerate(rb):
                    if qa + qs == qb and tjb in _fuse(tja, tjs):
                        keys.append((ia, s, ib))
                        dims.append((da, db))
        raw = block_data(keys, dims, seed, 100 + k)
        if k < center:        # left-canonical: orthonormalise per output sector
            for ib in range(len(rb)):
                ks = [key for key in keys if key[2] == ib]
                if not ks:
                    continue
                M = np.concatenate([raw[key] for key in ks], axis=0)
                Q, _ = np.linalg.qr(M)
                r = 0
                for key in ks:
                    n = raw[key].shape[0]
                    raw[key] = Q[r:r + n]
                    r += n
        elif k > center:      # right-canonical: orthonormalise rows per input sector
            for ia in range(len(lb)):
                ks = [key for key in keys if key[0] == ia]
                if not ks:
                    continue
                M = np.concatenate([raw[key] for key in ks], axis=1)
                Q, _ = np.linalg.qr(M.conj().T)
                Q = Q.conj().T
                c = 0
                for key in ks:
                    n = raw[key].shape[1]
                    raw[key] = Q[:, c:c + n]
                    c += n
        else:
            nrm = np.sqrt(sum(np.sum(np.abs(v) ** 2) for v in raw.values()))
            for key in raw:
                raw[key] = raw[key] / nrm
        sites[k - 1] = raw
    return bonds, sites


def u1_profile(chi, seed, nsites, spread=2.0, window=6, big=None):
    """Sectors [(sz2, N, d)] of a U(1) x U(1) bond with `nsites` sites to its
    left at half filling: N within +-window of nsites (0 <= N <= 2 nsites),
    2 S^z within +-window, N - 2 S^z even, |2 S^z| <= N; degeneracies
    proportional to exp(-((N - nsites)^2 + (2 S^z)^2) / (2 spread^2)) with a
    +-10 % log-normal jitter, rounded (largest remainder) to sum to chi.
    big: optionally raise the first sector's degeneracy to this value (a
    block spanning several tiles with a ragged tail)."""
    rng = _rng(seed, 5, chi, nsites)
    labels = [(sz, n) for n in range(max(0, nsites - window), min(2 * nsites, nsites + window) + 1)
              for sz in range(-window, window + 1) if (n - sz) % 2 == 0 and abs(sz) <= n]
    w = np.array([np.exp(-((n - nsites) ** 2 + sz ** 2) / (2 * spread ** 2)) for sz, n in labels])
    w = w * np.exp(0.1 * rng.standard_normal(len(w)))
    target = w * chi / w.sum()
    d = np.floor(target).astype(np.int64)
    rem = chi - int(d.sum())
    for i in np.argsort(-(target - d), kind="stable")[:rem]:
        d[i] += 1
    out = [(sz, n, int(di)) for (sz, n), di in zip(labels, d) if di > 0]
    if big is not None and out:
        out[0] = (out[0][0], out[0][1], int(big))
    return out


U1_LOCAL = [(0, 0), (1, 1), (-1, 1), (0, 2)]     # (2 S^z, N) of s = n_up + 2 n_dn


def _u1_count(n, sz2, nn):
    """Number of occupation states of n sites with 2 S^z = sz2 and N = nn."""
    from math import comb
    if (nn + sz2) % 2 or nn < 0:
        return 0
    nu, nd = (nn + sz2) // 2, (nn - sz2) // 2
    if nu < 0 or nd < 0 or nu > n or nd > n:
        return 0
    return comb(n, nu) * comb(n, nd)


def u1_random_mps(L, chi, seed, center=1, spread=2.0, window=6):
    """Random U(1) x U(1) MPS of L sites at half filling (2 S^z = 0, N = L) in
    mixed-canonical form with the centre on ``center``, the abelian analogue
    of ``random_mps``: bond k gets ``u1_profile(chi, ., k)`` capped sector by
    sector by the state counts of both sides and by the isometry condition of
    the neighbouring tensor.

    Returns (bonds, sites): bonds[k] = [(sz2, N, d)] for k = 0..L;
    sites[k-1] = {(ia, s, ib): d_a x d_b complex array}, s = 0..3."""
    bonds = [None] * (L + 1)
    bonds[0] = [(0, 0, 1)]
    bonds[L] = [(0, L, 1)]
    for k in range(1, L):
        bond = []
        for sz2, nn, d in u1_profile(chi, seed + 7919 * k, k, spread=spread, window=window):
            c = min(d, _u1_count(k, sz2, nn), _u1_count(L - k, -sz2, L - nn))
            if c > 0:
                bond.append((sz2, nn, c))
        bonds[k] = sorted(bond)
    for k in range(1, center):
        prev = bonds[k - 1]
        nb = []
        for sz2, nn, d in bonds[k]:
            rows = sum(da for (qa, na, da) in prev for qs, ns in U1_LOCAL if qa + qs == sz2 and na + ns == nn)
            if min(d, rows) > 0:
                nb.append((sz2, nn, min(d, rows)))
        bonds[k] = nb
    for k in range(L - 1, center - 1, -1):
        nxt = bonds[k + 1]
        nb = []
        for sz2, nn, d in bonds[k]:
            cols = sum(db for (qb, nb_, db) in nxt for qs, ns in U1_LOCAL if sz2 + qs == qb and nn + ns == nb_)
            if min(d, cols) > 0:
                nb.append((sz2, nn, min(d, cols)))
        bonds[k] = nb
    sites = [None] * L
    for k in range(1, L + 1):
        lb, rb = bonds[k - 1], bonds[k]
        keys, dims = [], []
        for ia, (qa, na, da) in enumerate(lb):
            for s, (qs, ns) in enumerate(U1_LOCAL):
                for ib, (qb, nb_, db) in enumerate(rb):
                    if qa + qs == qb and na + ns == nb_:
                        keys.append((ia, s, ib))
                        dims.append((da, db))
        raw = block_data(keys, dims, seed, 300 + k)
        if k < center:
            for ib in range(len(rb)):
                ks = [key for key in keys if key[2] == ib]
                if not ks:
                    continue
                Q, _ = np.linalg.qr(np.concatenate([raw[key] for key in ks], axis=0))
                r = 0
                for key in ks:
                    n = raw[key].shape[0]
                    raw[key] = Q[r:r + n]
                    r += n
        elif k > center:
            for ia in range(len(lb)):
                ks = [key for key in keys if key[0] == ia]
                if not ks:
                    continue
                Q, _ = np.linalg.qr(np.concatenate([raw[key] for key in ks], axis=1).conj().T)
                Q = Q.conj().T
                c = 0
                for key in ks:
                    n = raw[key].shape[1]
                    raw[key] = Q[:, c:c + n]
                    c += n
        else:
            nrm = np.sqrt(sum(np.sum(np.abs(v) ** 2) for v in raw.values()))
            for key in raw:
                raw[key] = raw[key] / nrm
        sites[k - 1] = raw
    return bonds, sites
