"""H_eff at the benchmark's full sizes: middle bond of an L = 60 chain at
chi = 4096 (Table-S2-shaped sectors), at chi = 16384 with a few hundred
log-normal uneven blocks, and at the late-time chi ~ 62 000 (Table-S2 shape:
a 9.4 GB two-site tensor and 6.2 GB of environments on one device), in the
launch configuration bench.py times.  The oracle cannot expand the whole problem, so sampled output blocks
are computed one by one on sector-restricted bonds (oracle.sampled) and
compared element by element; properties that hold at any size (linearity,
bit-reproducibility) cover the rest.  FP32 block products are checked
against the same oracle blocks at their stated tolerance."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2606_04771_amd as T
from oracle import sampled as S
import synth
from tests._harness import torch_stream_handle, pack, unpack

pytestmark = pytest.mark.gpu

L, SITE, t_h, U = 60, 30, 1.0, 4.0


def _profile(kind, seed):
    if kind == "table-s2-4096":     # the benchmark's middle bond
        return synth.sector_profile(4096, seed, parity=(SITE - 1) % 2)
    if kind == "table-s2-62000":    # the late-time segment's bond dimension
        return synth.sector_profile(62000, seed, parity=(SITE - 1) % 2)
    # a few hundred uneven blocks at chi = 16384: log-normal degeneracies
    return synth.lognormal_profile(16384, seed, (SITE - 1) % 2, qmax=4, tjmax=4)


def _build(kind):
    assert torch.cuda.is_available()
    left = _profile(kind, 7919 * (SITE - 1))
    right = _profile(kind, 7919 * (SITE + 1))
    bl, br = T.Bond(left), T.Bond(right)
    xk, xo, xt, xd = T.center_layout(bl, br, 2)
    lk, lo, lt, ld = T.env_layout(bl)
    rk, ro, rt, rd = T.env_layout(br)
    print(f"\n{kind}: {len(xk)} blocks, theta {xt * 16 / 1e9:.2f} GB, "
          f"environments {(lt + rt) * 16 / 1e9:.2f} GB; drawing inputs", flush=True)
    X = synth.block_data([tuple(k) for k in xk], xd, 21)
    nrm = np.sqrt(sum(np.sum(np.abs(v) ** 2) for v in X.values()))
    X = {k: v / nrm for k, v in X.items()}
    dev = {"x": torch.from_numpy(pack([X[tuple(k)] for k in xk], xo, xt)).to("cuda")}
    Lb = synth.block_data([tuple(k) for k in lk], ld, 22)
    dev["L"] = torch.from_numpy(pack([Lb[tuple(k)] for k in lk], lo, lt)).to("cuda")
    Rb = synth.block_data([tuple(k) for k in rk], rd, 23)
    dev["R"] = torch.from_numpy(pack([Rb[tuple(k)] for k in rk], ro, rt)).to("cuda")
    print(f"{kind}: inputs on the device", flush=True)
    ctx = T.Context(0, stream=torch_stream_handle())   # ordered with torch's work
    return dict(left=left, right=right, bl=bl, br=br, xk=xk, xo=xo, xt=xt, xd=xd, lk=lk, lo=lo, lt=lt,
                rk=rk, ro=ro, rt=rt, X=X, Lb=Lb, Rb=Rb, dev=dev, ctx=ctx)


@pytest.fixture(scope="module", params=["table-s2-4096", "lognormal-16384", "table-s2-62000"])
def problem(request):
    p = _build(request.param)
    yield p
    p["ctx"].close()
    del p["dev"]
    torch.cuda.empty_cache()


def _apply(p, x_dev, prec=T.FP64):
    y = torch.full_like(x_dev, float("nan"))
    p["ctx"].set_precision(prec)
    try:
        p["ctx"].heff_apply(T.Model(L, t_h, U), SITE, 2, p["bl"], p["br"],
                            T.Blocks(p["lk"], p["lo"], p["dev"]["L"].data_ptr(), p["lt"]),
                            T.Blocks(p["rk"], p["ro"], p["dev"]["R"].data_ptr(), p["rt"]),
                            T.Blocks(p["xk"], p["xo"], x_dev.data_ptr(), p["xt"]),
                            T.Blocks(p["xk"], p["xo"], y.data_ptr(), p["xt"]))
        p["ctx"].synchronize()
    finally:
        p["ctx"].set_precision(T.FP64)
    return y.cpu().numpy()


def _samples(p, n=10):
    """Output blocks small enough for the oracle, spread over the spectrum."""
    Lkeys = [tuple(int(v) for v in k) for k in p["lk"]]
    Rkeys = [tuple(int(v) for v in k) for k in p["rk"]]
    keys = [tuple(int(v) for v in k) for k in p["xk"]]
    sizes = [np.prod(S.restricted_dims(p["left"], p["right"], Lkeys, Rkeys, k)) for k in keys]
    order = np.argsort(sizes)
    ok = [keys[i] for i in order if sizes[i] <= 800_000]
    if len(ok) < 3:   # large blocks only (chi = 16384): the four smallest (~10 s of oracle each)
        return [keys[i] for i in order[:4]]
    idx = np.unique(np.linspace(0, len(ok) - 1, n).astype(int))
    return [ok[i] for i in idx]


def test_fullsize_heff_sampled_blocks_fp64_and_fp32(problem):
    p = problem
    y64 = _apply(p, p["dev"]["x"], T.FP64)
    y32 = _apply(p, p["dev"]["x"], T.FP32)
    yb3 = _apply(p, p["dev"]["x"], T.BF16X3)
    assert np.isfinite(y64).all()
    print(f"norm-wise vs FP64: fp32 {np.linalg.norm(y32 - y64) / np.linalg.norm(y64):.2e} "
          f"bf16x3 {np.linalg.norm(yb3 - y64) / np.linalg.norm(y64):.2e}", flush=True)
    ys64 = dict(zip([tuple(int(v) for v in k) for k in p["xk"]], unpack(y64, p["xo"], p["xd"])))
    ys32 = dict(zip([tuple(int(v) for v in k) for k in p["xk"]], unpack(y32, p["xo"], p["xd"])))
    ysb3 = dict(zip([tuple(int(v) for v in k) for k in p["xk"]], unpack(yb3, p["xo"], p["xd"])))
    worst64 = worst32 = worstb3 = 0.0
    for key in _samples(p):
        ref, dims = S.heff2_block(p["left"], p["right"], p["Lb"], p["Rb"], p["X"], key, SITE, t_h, U)
        scale = max(np.abs(ref).max(), 1e-300)
        e64 = np.abs(ys64[key] - ref).max() / scale
        e32 = np.abs(ys32[key] - ref).max() / scale
        eb3 = np.abs(ysb3[key] - ref).max() / scale
        print(f"block {key} dims {ref.shape} restricted {dims}: fp64 {e64:.2e} fp32 {e32:.2e} bf16x3 {eb3:.2e}",
              flush=True)
        worst64, worst32, worstb3 = max(worst64, e64), max(worst32, e32), max(worstb3, eb3)
    assert worst64 < 1e-12
    assert worst32 < 4e-6
    assert worstb3 < 4e-6


def test_fullsize_heff_linearity_and_determinism(problem):
    p = problem
    x = p["dev"]["x"]
    rng = np.random.default_rng(3)
    z = torch.from_numpy(rng.standard_normal(x.shape[0]) + 1j * rng.standard_normal(x.shape[0])).to("cuda")
    a, b = 0.3 - 0.7j, -1.1 + 0.2j
    y1 = _apply(p, x)
    y2 = _apply(p, z)
    y3 = _apply(p, a * x + b * z)
    err = np.abs(y3 - (a * y1 + b * y2)).max() / np.abs(y3).max()
    assert err < 1e-13
    assert np.array_equal(_apply(p, x), y1)


def _chains(p):
    """K-chain depth of every output block (sum of the K of its block
    products) from the exported host plan, and the output keys."""
    Lk = T.Blocks(p["lk"], p["lo"], 0, p["lt"])
    Rk = T.Blocks(p["rk"], p["ro"], 0, p["rt"])
    Xk = T.Blocks(p["xk"], p["xo"], 0, p["xt"])
    terms, _ = T.heff_plan(T.Model(L, t_h, U), SITE, 2, p["bl"], p["br"], Lk, Rk, Xk)
    chain = np.zeros(len(p["xk"]), np.int64)
    for kind, out, inn, env, coef in terms:
        if kind == 0:
            chain[out] += p["xd"][inn][0]
        elif kind == 1:
            chain[out] += p["xd"][inn][1]
    return chain, [tuple(int(v) for v in k) for k in p["xk"]]


def _cross_cost(p, key):
    """Rough flop count of the inclusion-exclusion oracle for one block."""
    lconn = {key[0]} | {k[2] for k in (tuple(int(v) for v in kk) for kk in p["lk"]) if k[0] == key[0]}
    rconn = {key[4]} | {k[2] for k in (tuple(int(v) for v in kk) for kk in p["rk"]) if k[0] == key[4]}
    full = lambda b, S_: sum(b[i][2] * (b[i][1] + 1) for i in S_)
    l1, r1 = full(p["left"], lconn), full(p["right"], {key[4]})
    l2, r2 = full(p["left"], {key[0]}), full(p["right"], rconn)
    return l1 * l1 * r1 + r2 * r2 * l2


@pytest.fixture(scope="module")
def p4096():
    p = _build("table-s2-4096")
    yield p
    p["ctx"].close()


@pytest.fixture(scope="module")
def p16384():
    p = _build("lognormal-16384")
    yield p
    p["ctx"].close()


def test_fullsize_longest_k_chain_block(p4096):
    """The output block with the longest K chain of the chi = 4096 apply (the
    tile that runs longest in the benchmark's launch), against the oracle."""
    p = p4096
    chain, keys = _chains(p)
    o = int(np.argmax(chain))
    key = keys[o]
    print(f"longest chain {chain[o]} (median {int(np.median(chain))}) at block {key} {p['xd'][o]}", flush=True)
    ref = S.heff2_block_cross(p["left"], p["right"], p["Lb"], p["Rb"], p["X"], key, SITE, t_h, U)
    scale = np.abs(ref).max()
    for prec, tol in ((T.FP64, 1e-12), (T.FP32, 4e-6), (T.BF16X3, 4e-6)):
        y = _apply(p, p["dev"]["x"], prec)
        got = unpack(y, [p["xo"][o]], [p["xd"][o]])[0]
        err = np.abs(got - ref).max() / scale
        print(f"  prec {prec}: {err:.2e}", flush=True)
        assert err < tol


def test_fullsize_split_k_chains_match_the_oracle(p16384):
    """chi = 16384: K chains split on request (tdvp_ctx_set_split with a cap of
    0.1 x the mean work per resident workgroup, pieces >= 64 deep) and summed by
    the second kernel.  The default rule splits no tile at this shape (no tile
    reaches its cap), so the split launch is forced here.  The blocks whose bits
    differ from an unsplit launch are the split ones; there must be some, the
    two launches must agree to rounding, and the cheapest split block with a
    long chain must match the oracle."""
    p = p16384
    ctx = p["ctx"]
    ctx.set_split(0.1, 64)
    try:
        y_split = _apply(p, p["dev"]["x"])
        ctx.set_split(0.0, 128)
        y_plain = _apply(p, p["dev"]["x"])
    finally:
        ctx.set_split()
    assert np.abs(y_split - y_plain).max() <= 1e-13 * np.abs(y_plain).max()
    chain, keys = _chains(p)
    ys = unpack(y_split, p["xo"], p["xd"])
    yp = unpack(y_plain, p["xo"], p["xd"])
    split = [o for o in range(len(keys)) if not np.array_equal(ys[o], yp[o])]
    print(f"{len(split)} of {len(keys)} output blocks computed from split chains", flush=True)
    assert split
    long_ = [o for o in split if chain[o] >= np.percentile(chain, 75)]
    assert long_
    o = min(long_, key=lambda i: _cross_cost(p, keys[i]))
    key = keys[o]
    print(f"checking split block {key} {p['xd'][o]} chain {chain[o]}", flush=True)
    ref = S.heff2_block_cross(p["left"], p["right"], p["Lb"], p["Rb"], p["X"], key, SITE, t_h, U)
    err = np.abs(ys[o] - ref).max() / np.abs(ref).max()
    print(f"  fp64 split: {err:.2e}", flush=True)
    assert err < 1e-12
