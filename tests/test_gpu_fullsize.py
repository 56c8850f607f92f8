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


@pytest.fixture(scope="module", params=["table-s2-4096", "lognormal-16384", "table-s2-62000"])
def problem(request):
    assert torch.cuda.is_available()
    left = _profile(request.param, 7919 * (SITE - 1))
    right = _profile(request.param, 7919 * (SITE + 1))
    bl, br = T.Bond(left), T.Bond(right)
    xk, xo, xt, xd = T.center_layout(bl, br, 2)
    lk, lo, lt, ld = T.env_layout(bl)
    rk, ro, rt, rd = T.env_layout(br)
    print(f"\n{request.param}: {len(xk)} blocks, theta {xt * 16 / 1e9:.2f} GB, "
          f"environments {(lt + rt) * 16 / 1e9:.2f} GB; drawing inputs", flush=True)
    X = synth.block_data([tuple(k) for k in xk], xd, 21)
    nrm = np.sqrt(sum(np.sum(np.abs(v) ** 2) for v in X.values()))
    X = {k: v / nrm for k, v in X.items()}
    dev = {"x": torch.from_numpy(pack([X[tuple(k)] for k in xk], xo, xt)).to("cuda")}
    Lb = synth.block_data([tuple(k) for k in lk], ld, 22)
    dev["L"] = torch.from_numpy(pack([Lb[tuple(k)] for k in lk], lo, lt)).to("cuda")
    Rb = synth.block_data([tuple(k) for k in rk], rd, 23)
    dev["R"] = torch.from_numpy(pack([Rb[tuple(k)] for k in rk], ro, rt)).to("cuda")
    print(f"{request.param}: inputs on the device", flush=True)
    ctx = T.Context(0, stream=torch_stream_handle())   # ordered with torch's work
    yield dict(left=left, right=right, bl=bl, br=br, xk=xk, xo=xo, xt=xt, xd=xd, lk=lk, lo=lo, lt=lt,
               rk=rk, ro=ro, rt=rt, X=X, Lb=Lb, Rb=Rb, dev=dev, ctx=ctx)
    ctx.close()


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
    assert worst32 < 2e-5
    assert worstb3 < 2e-5


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
