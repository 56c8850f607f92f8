"""Allocation-free environment update (tdvp_env_update_noalloc) against the
allocating entry point tdvp_env_update, through the C ABI.

Two calls in a row on one context, the second smaller (a chi = 4096 bond
with Table-S2-shaped sectors, then a chi = 120 one), in FP64 and in FP32:
each output must be bit-identical to tdvp_env_update's on the same inputs,
since both run the same kernels on the same programs.  The context's allocator counts its
calls: the allocation-free calls must make none.  An update whose stage-1
products exceed the static array returns NOMEM and launches nothing."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2606_04771_amd as T
import synth
from tests._harness import torch_stream_handle, pack

pytestmark = pytest.mark.gpu

t_h, U = 1.0, 4.0


def _case(bond_left, bond_right, site, direction, seed, random=True):
    """Inputs of one environment update at `site` (bond_left = bond site-1,
    bond_right = bond site); zero data when random is False."""
    if direction > 0:
        bin_, bout = bond_left, bond_right
        tk, to, tt, td = T.center_layout(T.Bond(bin_), T.Bond(bout), 1)
    else:
        bin_, bout = bond_right, bond_left
        tk, to, tt, td = T.center_layout(T.Bond(bout), T.Bond(bin_), 1)
    bi, bo = T.Bond(bin_), T.Bond(bout)
    ek, eo, et, ed = T.env_layout(bi)
    ok, oo, ot, od = T.env_layout(bo)
    if random:
        ts = synth.block_data([tuple(k) for k in tk], td, seed)
        Es = synth.block_data([tuple(k) for k in ek], ed, seed + 1)
        t_d = torch.from_numpy(pack([ts[tuple(k)] for k in tk], to, tt)).to("cuda")
        e_d = torch.from_numpy(pack([Es[tuple(k)] for k in ek], eo, et)).to("cuda")
    else:
        t_d = torch.zeros(max(tt, 1), dtype=torch.complex128, device="cuda")
        e_d = torch.zeros(max(et, 1), dtype=torch.complex128, device="cuda")
    return dict(bi=bi, bo=bo, tk=tk, to=to, tt=tt, ek=ek, eo=eo, et=et, ok=ok, oo=oo, ot=ot, t_d=t_d, e_d=e_d)


def _run(ctx, c, site, direction, noalloc):
    out = torch.full((max(c["ot"], 1),), float("nan"), dtype=torch.complex128, device="cuda")
    f = ctx.env_update_noalloc if noalloc else ctx.env_update
    f(T.Model(60, t_h, U), site, direction, c["bi"], c["bo"], T.Blocks(c["ek"], c["eo"], c["e_d"].data_ptr(), c["et"]),
      T.Blocks(c["tk"], c["to"], c["t_d"].data_ptr(), c["tt"]), T.Blocks(c["ok"], c["oo"], out.data_ptr(), c["ot"]))
    ctx.synchronize()
    return out.cpu().numpy()


@pytest.fixture(scope="module")
def counted():
    """A context whose device allocator (torch's caching allocator) counts
    its calls."""
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    stream = torch_stream_handle()
    calls = []

    def alloc(n, user):
        calls.append(int(n))
        return torch.cuda.caching_allocator_alloc(int(n), 0, int(stream))

    def free(p, user):
        torch.cuda.caching_allocator_delete(int(p))

    cbs = (T._ALLOC_FN(alloc), T._FREE_FN(free))
    ctx = T.Context(0, stream=stream, allocator=cbs)
    yield ctx, calls
    ctx.close()


@pytest.mark.parametrize("prec", [T.FP64, T.FP32])
def test_noalloc_env_update_matches_the_allocating_call(counted, prec):
    ctx, calls = counted
    site = 30
    big = _case(synth.sector_profile(4096, 11, parity=(site - 1) % 2),
                synth.sector_profile(4096, 12, parity=site % 2), site, +1 if prec == T.FP64 else -1, 13)
    small = _case(synth.sector_profile(120, 21, parity=(site - 1) % 2),
                  synth.sector_profile(120, 22, parity=site % 2), site, -1 if prec == T.FP64 else +1, 23)
    dirs = (+1, -1) if prec == T.FP64 else (-1, +1)
    ctx.set_precision(prec)
    try:
        print(f"prec {prec}: chi=4096 dir {dirs[0]:+d}, then chi=120 dir {dirs[1]:+d}", flush=True)
        n0 = len(calls)
        got_big = _run(ctx, big, site, dirs[0], True)
        got_small = _run(ctx, small, site, dirs[1], True)
        assert len(calls) == n0, f"allocation-free calls allocated {calls[n0:]}"
        ref_big = _run(ctx, big, site, dirs[0], False)
        ref_small = _run(ctx, small, site, dirs[1], False)
        # once more after the allocating calls, which left their own programs cached
        again_small = _run(ctx, small, site, dirs[1], True)
    finally:
        ctx.set_precision(T.FP64)
    for got, ref in ((got_big, ref_big), (got_small, ref_small), (again_small, ref_small)):
        assert np.isfinite(ref).all()
        assert np.array_equal(got, ref)
    print(f"  bit-identical; {big['ot']} and {small['ot']} output elements", flush=True)


def test_noalloc_env_update_beyond_the_static_array(counted):
    """chi = 16384 (stage-1 products ~0.5 GB): NOMEM, output untouched."""
    ctx, calls = counted
    site = 30
    lp = (site - 1) % 2
    c = _case(synth.lognormal_profile(16384, 31, lp, qmax=4, tjmax=4),
              synth.lognormal_profile(16384, 32, 1 - lp, qmax=4, tjmax=4), site, +1, 33, random=False)
    out = torch.full((c["ot"],), float("nan"), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(T.TdvpError) as e:
        ctx.env_update_noalloc(T.Model(60, t_h, U), site, +1, c["bi"], c["bo"],
                               T.Blocks(c["ek"], c["eo"], c["e_d"].data_ptr(), c["et"]),
                               T.Blocks(c["tk"], c["to"], c["t_d"].data_ptr(), c["tt"]),
                               T.Blocks(c["ok"], c["oo"], out.data_ptr(), c["ot"]))
    assert e.value.code == -4 and "static scratch" in str(e.value)
    ctx.synchronize()
    assert torch.isnan(out).all().item()
