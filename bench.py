#!/usr/bin/env python3
"""Benchmark of the two-site TDVP hot path on one MI355X.

Workload (synthetic, seeded): an L = 60 Fermi-Hubbard chain (t = 1,
U = 4) in U(1)xSU(2)-reduced MPS form with every interior bond at full-state
bond dimension chi = 4096, sector degeneracies shaped like the paper's
Table S2.  Two measurements, both with all data resident in HBM:

* H_eff.Theta: the effective Hamiltonian of the middle sites (30, 31)
  applied to a random normalised two-site tensor, environments built on the
  GPU from a random mixed-canonical MPS.  Per-launch duration from HIP events
  on the library's stream; throughput = algorithmic flops (8 per complex
  multiply-add of every nonzero block product) / duration.
* One step = one full two-site TDVP sweep (dt = 0.05, discarded-weight
  tolerance 1e-4, chi cap 4096) of a seeded random chi = 4096 MPS: every
  bond merged, Krylov-evolved, split by SVD, environments updated, centre
  evolved back.  Reported as s/sweep.
* Mixed precision: the same applies with FP32 block products (error against
  the FP64 apply), and a second run of the same sweeps from the same initial
  state with FP32 block products in H_eff and the environment updates (FP64
  Lanczos, SVD and gauge shifts): its s/sweep, the state error
  |psi_64 - psi_mixed| after the first and after the last sweep (from MPS
  overlaps), and the largest deviation of the site-resolved <S^z> and
  double occupancy.
* Larger bonds (context, not the headline): H_eff.Theta at chi = 16384 with
  a few hundred log-normal uneven blocks (grouped launch against one launch
  per output block), and at the late-time chi ~ 62 000 (a 9.4 GB two-site
  tensor), per precision; one-site sweeps on the saturated state.

Prints one JSON line.  ``--gpus N`` with N > 1 is refused: the library runs
on a single GPU.
"""
import argparse
import json
import os
import sys
import time

METRIC = "H_eff·Θ TFLOP/s + s/sweep at L=60 χ=4096; mixed vs FP64 at ≤1e-4 obs err"
# MI355X dense matrix-core peaks (TFLOP/s).  Split-BF16 products issue six
# bf16 slice products per logical real product, so their logical-flop
# ceiling is the bf16 peak / 6.
BF16_PEAK = 2516.0
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": BF16_PEAK / 6}


def rooflines(by_prec):
    """Fraction of each precision's matrix-core ceiling reached by the H_eff
    applies (logical flops: 8 per complex multiply-add)."""
    out = {}
    for name, r in by_prec.items():
        if name not in PEAK or "tflops" not in r:
            continue
        out[name] = {"achieved": r["tflops"], "peak": PEAK[name], "unit": "TFLOP/s",
                     "frac": r["tflops"] / PEAK[name], "traffic": measured_traffic(name)}
        if name == "bf16x3":
            out[name]["bf16_issue_frac"] = 6 * r["tflops"] / BF16_PEAK
    return out


def restore_env(name, value):
    if value is None:
        os.environ.pop(name, None)
    else:
        os.environ[name] = value


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def pack(blocks, keys, offs, total):
    import numpy as np
    buf = np.zeros(max(total, 1), np.complex128)
    for k, o in zip(keys, offs):
        a = blocks[tuple(int(v) for v in k)]
        buf[o:o + a.size] = a.reshape(-1, order="F")
    return buf


def measured_traffic(prec):
    """HBM bytes per H_eff launch of the given precision's kernel at the
    chi = 4096 middle bond, from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a
    plain copy of known size), or None when the kernel sources changed since
    the counters were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", f"heff_gemm_{prec}_chi4096_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in ("gemm.hip", "ctx.hpp", "capi_dev.cpp", "plan.cpp"):
        with open(os.path.join(here, "paper_2606_04771_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return rec["bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def large_heff(args, T, torch, stream, ctx, model, late=False):
    """H_eff.Theta at the middle bond of L = 60 with large, uneven blocks.

    Default: chi = 16384 (full-state units), a few hundred sector blocks with
    degeneracies log-normal (median 200, sigma 1) over the labels |q| <= 4,
    2j <= 4, clipped to [8, 2048], rescaled to chi; environments and Theta
    complex normal (numpy, seeded); FP64, FP32 and split-BF16 grouped
    launches, and FP64 with one launch per output block.
    late=True: the late-time bond dimension chi ~ 62 000 with Table-S2-shaped
    sectors (a 9.4 GB two-site tensor); operands drawn on the device (seeded
    torch generator: only throughput is measured here, the full-size tests
    check the values), grouped launches only."""
    import numpy as np
    import synth
    site = 30
    if late:
        chi = 62000
        left = synth.sector_profile(chi, 7919 * (site - 1), parity=1)
        right = synth.sector_profile(chi, 7919 * (site + 1), parity=1)
        label = f"chi={chi} L=60 middle bond, Table-S2-shaped sectors (late-time segment)"
    else:
        chi = 16384
        left = synth.lognormal_profile(chi, 7919 * (site - 1), 1, qmax=4, tjmax=4)
        right = synth.lognormal_profile(chi, 7919 * (site + 1), 1, qmax=4, tjmax=4)
        label = (f"chi={chi} L=60 middle bond, log-normal sector dims (median 200, sigma 1, |q|<=4, "
                 f"2j<=4, clipped 8..2048, rescaled)")
    bl, br = T.Bond(left), T.Bond(right)
    xk, xo, xt, xd = T.center_layout(bl, br, 2)
    lk, lo, lt, ld = T.env_layout(bl)
    rk, ro, rt, rd = T.env_layout(br)
    if late:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(args.seed + 62)
        draw = lambda n: torch.randn(max(n, 1), dtype=torch.complex128, device="cuda", generator=gen)
        x_d, L_d, R_d = draw(xt), draw(lt), draw(rt)
        x_d /= torch.linalg.vector_norm(x_d)
    else:
        dev = lambda a: torch.from_numpy(a).to("cuda")
        X = synth.block_data([tuple(k) for k in xk], xd, args.seed + 31, 13)
        Lb = synth.block_data([tuple(k) for k in lk], ld, args.seed + 32, 14)
        Rb = synth.block_data([tuple(k) for k in rk], rd, args.seed + 33, 15)
        x_d = dev(pack(X, xk, xo, xt))
        L_d = dev(pack(Lb, lk, lo, lt))
        R_d = dev(pack(Rb, rk, ro, rt))
        del X, Lb, Rb
    y_d = torch.zeros_like(x_d)
    torch.cuda.synchronize()
    Lbk = T.Blocks(lk, lo, L_d.data_ptr(), lt)
    Rbk = T.Blocks(rk, ro, R_d.data_ptr(), rt)
    xb = T.Blocks(xk, xo, x_d.data_ptr(), xt)
    yb = T.Blocks(xk, xo, y_d.data_ptr(), xt)
    _, flops = T.heff_plan(model, site, 2, bl, br, Lbk, Rbk, xb)

    def timed(p, warm, reps):
        ctx.set_precision(p)
        for _ in range(warm):
            ctx.heff_apply(model, site, 2, bl, br, Lbk, Rbk, xb, yb)
        ctx.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            ctx.heff_apply(model, site, 2, bl, br, Lbk, Rbk, xb, yb)
        b.record(stream)
        ctx.synchronize()
        return a.elapsed_time(b) * 1e-3 / reps

    res = {"workload": label, "blocks": len(xk), "theta_elems": int(xt),
           "theta_gb": round(xt * 16 / 1e9, 2), "env_gb": round((lt + rt) * 16 / 1e9, 2),
           "block_dim_max": int(max(r for r, c in xd)), "flops_per_apply": flops}
    # FP64 warm-up covers the tiling autotuner's measured launches
    runs = (("fp64", T.FP64, 11, 3), ("fp32", T.FP32, 1, 3), ("bf16x3", T.BF16X3, 1, 3)) if late else \
        (("fp64", T.FP64, 12, 10), ("fp32", T.FP32, 10, 10), ("bf16x3", T.BF16X3, 10, 10))
    for name, p, warm, reps in runs:
        dt = timed(p, warm, reps)
        res[name] = {"ms_per_apply": 1e3 * dt, "tflops": flops / dt / 1e12}
        print(f"bench: chi={chi} H_eff {name} {1e3 * dt:.2f} ms, {flops / dt / 1e12:.2f} TFLOP/s",
              file=sys.stderr, flush=True)
    res["roofline_by_precision"] = rooflines({k: res[k] for k in ("fp64", "fp32", "bf16x3")})
    for mode, key in ((2, "fp64_dispatcher_grid"), (3, "fp64_persistent_grid"), (4, "fp64_wave_tiles")):
        before = os.environ.get("TDVP_FORCE_TILING")
        os.environ["TDVP_FORCE_TILING"] = str(mode)
        try:
            dt = timed(T.FP64, 2, 3 if late else 10)
        finally:
            restore_env("TDVP_FORCE_TILING", before)
        res[key] = {"ms_per_apply": 1e3 * dt, "tflops": flops / dt / 1e12}
        print(f"bench: chi={chi} H_eff fp64 tiling mode {mode}, {key}: {1e3 * dt:.2f} ms", file=sys.stderr, flush=True)
    if not late:
        os.environ["TDVP_PER_BLOCK"] = "1"
        try:
            dt = timed(T.FP64, 2, 3)
        finally:
            del os.environ["TDVP_PER_BLOCK"]
        res["fp64_one_launch_per_block"] = {"ms_per_apply": 1e3 * dt, "tflops": flops / dt / 1e12,
                                            "launches_per_apply": len(xk)}
        print(f"bench: chi={chi} H_eff fp64, one launch per output block: {1e3 * dt:.2f} ms, "
              f"{flops / dt / 1e12:.2f} TFLOP/s", file=sys.stderr, flush=True)
    if late and args.late_bond:
        # the other two costs of one bond update at this size, with the memory
        # plan's complex64 Krylov basis: a fixed-length Krylov exponential
        # (tol 0) and the split of Theta (operands are random, so only the
        # times and the device memory are meaningful here)
        ctx.set_precision(T.FP64)
        ctx.set_krylov_storage(T.FP32)
        ctx.memory(reset_peak=True)
        m = args.late_bond
        torch.cuda.synchronize()
        t0 = time.time()
        rc, info = ctx.krylov_expm(model, site, 2, bl, br, Lbk, Rbk, xb, -0.025j, tol=0.0, maxdim=m, check=False)
        t_kry = time.time() - t0
        ctx.set_krylov_storage(T.FP64)
        print(f"bench: chi={chi} Krylov exponential, {info['iters']} iterations (complex64 basis): {t_kry:.2f} s",
              file=sys.stderr, flush=True)
        x_d /= torch.linalg.vector_norm(x_d)
        torch.cuda.synchronize()
        t0 = time.time()
        out, sv, disc = ctx.split(bl, br, xb, +1, eps_tol=1e-8, chi_cap=10 ** 6)
        t_split = time.time() - t0
        bond = out.bond(1)
        out.close()
        print(f"bench: chi={chi} split: {t_split:.2f} s, {len(sv)} sectors, largest sector matrix side "
              f"{max(min(len(v), 10 ** 9) for v in sv.values())}", file=sys.stderr, flush=True)
        res["bond_update"] = {"krylov_iterations": int(info["iters"]), "krylov_s": t_kry,
                              "krylov_s_per_iteration": t_kry / max(info["iters"], 1), "split_s": t_split,
                              "split_sectors": len(sv), "kept_reduced_dim": int(sum(d for _, _, d in bond)),
                              "peak_device_gb": ctx.memory()[1] / 1e9}
    ctx.set_precision(T.FP64 if args.prec == "fp64" else T.FP32)
    del x_d, y_d, L_d, R_d
    torch.cuda.empty_cache()
    return res


def u1_heff(args, T, torch, stream, ctx, model, chi):
    """H_eff.Theta of the abelian U(1) x U(1) variant at the middle bond of
    L = 60 with the same full-state bond dimension: sectors (N, 2S^z) around
    half filling (synth.u1_profile), environments and Theta complex normal;
    FP64 and FP32 block products."""
    import numpy as np
    import synth
    site = 30
    left = synth.u1_profile(chi, 7919 * (site - 1), site - 1)
    right = synth.u1_profile(chi, 7919 * (site + 1), site + 1)
    bl, br = T.Bond(left), T.Bond(right)
    xk, xo, xt, xd = T.center_layout(bl, br, 2, abelian=True)
    lk, lo, lt, ld = T.env_layout(bl, abelian=True)
    rk, ro, rt, rd = T.env_layout(br, abelian=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(args.seed + 71)
    draw = lambda n: torch.randn(max(n, 1), dtype=torch.complex128, device="cuda", generator=gen)
    x_d, L_d, R_d = draw(xt), draw(lt), draw(rt)
    y_d = torch.zeros_like(x_d)
    torch.cuda.synchronize()
    Lb = T.Blocks(lk, lo, L_d.data_ptr(), lt)
    Rb = T.Blocks(rk, ro, R_d.data_ptr(), rt)
    xb = T.Blocks(xk, xo, x_d.data_ptr(), xt)
    yb = T.Blocks(xk, xo, y_d.data_ptr(), xt)
    _, flops = T.heff_plan(model, site, 2, bl, br, Lb, Rb, xb, abelian=True)
    res = {"workload": f"chi={chi} L=60 middle bond, U(1)xU(1) sectors (N, 2Sz) around half filling",
           "sectors": len(left), "blocks": len(xk), "theta_elems": int(xt), "flops_per_apply": flops}
    for name, p, warm, reps in (("fp64", T.FP64, 12, 10), ("fp32", T.FP32, 5, 10)):
        ctx.set_precision(p)
        for _ in range(warm):
            ctx.heff_apply(model, site, 2, bl, br, Lb, Rb, xb, yb, abelian=True)
        ctx.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            ctx.heff_apply(model, site, 2, bl, br, Lb, Rb, xb, yb, abelian=True)
        b.record(stream)
        ctx.synchronize()
        dt = a.elapsed_time(b) * 1e-3 / reps
        res[name] = {"ms_per_apply": 1e3 * dt, "tflops": flops / dt / 1e12}
        print(f"bench: U(1)xU(1) chi={chi} H_eff {name} {1e3 * dt:.2f} ms, {flops / dt / 1e12:.2f} TFLOP/s",
              file=sys.stderr, flush=True)
    ctx.set_precision(T.FP64 if args.prec == "fp64" else T.FP32)
    del x_d, y_d, L_d, R_d
    torch.cuda.empty_cache()
    return res


def u1_sweep(args, T, torch, stream, ctx, model, chi, run):
    """Two-site sweeps of the abelian U(1) x U(1) variant on a seeded random
    L = 60 MPS at the same full-state bond dimension (synth.u1_random_mps:
    sectors (2S^z, N) around half filling), with the run parameters of the
    U(1) x SU(2) sweep; the first sweep is untimed."""
    import synth
    L = model.L
    t0 = time.time()
    bonds, sites = synth.u1_random_mps(L, chi, args.seed + 200)
    print(f"bench: U(1)xU(1) random MPS built on the host in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    Tb = [T.Bond(b) for b in bonds]
    bufs, descs = [], []
    for k in range(1, L + 1):
        tk, to, tt, _ = T.center_layout(Tb[k - 1], Tb[k], 1, abelian=True)
        d = torch.from_numpy(pack(sites[k - 1], tk, to, tt)).to("cuda")
        bufs.append(d)
        descs.append(T.Blocks(tk, to, d.data_ptr(), tt))
    ctx.set_precision(T.FP64)
    mps = T.MPS.from_blocks(ctx, model, Tb, descs, abelian=True)
    torch.cuda.synchronize()
    del bufs, descs
    ctx.memory(reset_peak=True)
    infos = []
    for st in range(2):
        info = mps.sweep(**run)
        infos.append(info)
        print(f"bench: U(1)xU(1) sweep {st + 1}: {info['seconds']:.2f} s (lanczos {info['t_lanczos']:.2f}, "
              f"svd {info['t_svd']:.2f}, env {info['t_env']:.2f}), chi {info['max_chi']}, "
              f"krylov {info['krylov_iters']}", file=sys.stderr, flush=True)
    i = infos[-1]
    res = {"workload": f"L={L} U(1)xU(1) random MPS, chi={chi}, sectors (2Sz, N) around half filling; "
                       "dt=0.05, eps_tol=1e-4, chi cap, FP64",
           "s_per_sweep": i["seconds"], "sweep_phase_s": {k: i[k] for k in ("t_lanczos", "t_svd", "t_env")},
           "krylov_iters": int(i["krylov_iters"]), "heff_flops": i["heff_flops"],
           "lanczos_tflops": i["heff_flops"] / i["t_lanczos"] / 1e12 if i["t_lanczos"] > 0 else None,
           "max_chi": int(i["max_chi"]), "max_discarded": i["max_discarded"],
           "peak_device_gb": ctx.memory()[1] / 1e9, "sweeps": len(infos), "timed": 1}
    mps.close()
    ctx.set_precision(T.FP64 if args.prec == "fp64" else T.FP32)
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed sweeps")
    ap.add_argument("--warmup", type=int, default=1, help="untimed sweeps")
    ap.add_argument("--L", type=int, default=60)
    ap.add_argument("--chi", type=int, default=4096)
    ap.add_argument("--prec", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--heff-reps", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison run")
    ap.add_argument("--one-site-steps", type=int, default=2, help="one-site sweeps timed after the two-site ones")
    ap.add_argument("--no-large", action="store_true", help="skip the chi=16384 grouped-vs-per-block measurement")
    ap.add_argument("--no-late", action="store_true", help="skip the chi~62000 H_eff throughput measurement")
    ap.add_argument("--late-bond", type=int, default=8,
                    help="Krylov iterations of the timed chi~62000 bond update (Krylov exponential and split; 0: skip)")
    ap.add_argument("--no-abelian", action="store_true", help="skip the U(1)xU(1) H_eff and sweep measurements")
    ap.add_argument("--krylov-probe", type=int, default=0,
                    help="only run Krylov exponentials of exactly this many iterations at the middle bond "
                         "(Lanczos vector-kernel profile)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB three times (reference for the HBM byte counters)")
    args = ap.parse_args()
    # HIP's default of four hardware queues unless the caller chose otherwise
    # (read once, when HIP starts: before torch is imported); the split plans
    # its eigensolves per queue and measured fastest with four
    os.environ.setdefault("GPU_MAX_HW_QUEUES", "4")
    if args.copy_calibration:
        import torch
        n = 2 ** 26                       # 64 Mi complex128 = 1 GiB
        x = torch.ones(n, dtype=torch.complex128, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 3 * n * 16, "copy_bytes_written": 3 * n * 16}))
        return
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2606_04771_amd as T
    import synth

    L, chi, t_h, U = args.L, args.chi, 1.0, 4.0
    prec = T.FP64 if args.prec == "fp64" else T.FP32
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)   # torch's work and the library's are ordered on one stream
    ctx = T.Context(0, stream=stream.cuda_stream, precision=prec)
    model = T.Model(L, t_h, U)
    dev = lambda a: torch.from_numpy(a).to("cuda")

    # ---- H_eff at the middle bond ------------------------------------------------
    site = L // 2
    bonds, sites = synth.random_mps(L, chi, args.seed, center=site)
    Tb = [T.Bond(b) for b in bonds]
    keep = []

    def env_chain(direction):
        b0 = Tb[0] if direction > 0 else Tb[L]
        ek, eo, et, ed = T.env_layout(b0)
        env = torch.zeros(max(et, 1), dtype=torch.complex128, device="cuda")
        desc = (ek, eo, et)
        ks = range(1, site) if direction > 0 else range(L, site + 1, -1)
        for k in ks:
            bi, bo = (Tb[k - 1], Tb[k]) if direction > 0 else (Tb[k], Tb[k - 1])
            tk, to, tt, _ = T.center_layout(Tb[k - 1], Tb[k], 1)
            t_d = dev(pack(sites[k - 1], tk, to, tt))
            ok, oo, ot, _ = T.env_layout(bo)
            out = torch.zeros(max(ot, 1), dtype=torch.complex128, device="cuda")
            with torch.cuda.stream(stream):
                ctx.env_update(model, k, direction, bi, bo, T.Blocks(desc[0], desc[1], env.data_ptr(), desc[2]),
                               T.Blocks(tk, to, t_d.data_ptr(), tt), T.Blocks(ok, oo, out.data_ptr(), ot))
            keep.append((env, t_d))
            env, desc = out, (ok, oo, ot)
        ctx.synchronize()
        return env, desc

    torch.cuda.synchronize()
    t0 = time.time()
    Lenv, Ld = env_chain(+1)
    Renv, Rd = env_chain(-1)
    t_env_chain = time.time() - t0
    del keep[:]
    left, right = Tb[site - 1], Tb[site + 1]
    xk, xo, xt, xd = T.center_layout(left, right, 2)
    xs = synth.block_data([tuple(k) for k in xk], xd, args.seed + 1, 9)
    nrm = np.sqrt(sum(np.sum(np.abs(v) ** 2) for v in xs.values()))
    xs = {k: v / nrm for k, v in xs.items()}
    x_d = dev(pack(xs, xk, xo, xt))
    y_d = torch.zeros_like(x_d)
    Lb = T.Blocks(Ld[0], Ld[1], Lenv.data_ptr(), Ld[2])
    Rb = T.Blocks(Rd[0], Rd[1], Renv.data_ptr(), Rd[2])
    xb = T.Blocks(xk, xo, x_d.data_ptr(), xt)
    yb = T.Blocks(xk, xo, y_d.data_ptr(), xt)
    terms, flops = T.heff_plan(model, site, 2, left, right, Lb, Rb, xb)

    def time_applies(p):
        ctx.set_precision(p)
        for _ in range(12):   # includes the autotuner's measured launches (5 candidates x 2)
            ctx.heff_apply(model, site, 2, left, right, Lb, Rb, xb, yb)
        ctx.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.heff_reps)]
        for a, b in evs:
            a.record(stream)
            ctx.heff_apply(model, site, 2, left, right, Lb, Rb, xb, yb)
            b.record(stream)
        ctx.synchronize()
        d = np.array([a.elapsed_time(b) * 1e-3 for a, b in evs])
        return d, y_d.cpu().numpy()

    if args.krylov_probe:
        # Lanczos vector kernels at a fixed size: exponentials of exactly
        # krylov_probe iterations (tol 0) on the middle-bond problem, graph
        # replay on; the per-kernel durations come from a kernel trace of
        # this mode.
        m = args.krylov_probe
        ctx.set_precision(T.FP64)
        t_it = []
        for rep in range(4):
            x_d.copy_(dev(pack(xs, xk, xo, xt)))
            torch.cuda.synchronize()
            t0 = time.time()
            rc, info = ctx.krylov_expm(model, site, 2, left, right, Lb, Rb, xb, -0.025j, tol=0.0, maxdim=m,
                                       check=False)
            t_it.append((time.time() - t0) / max(info["iters"], 1))
            print(f"bench: krylov probe {rep}: {info['iters']} iterations ({info['graph_iters']} replayed), "
                  f"{1e3 * t_it[-1]:.3f} ms per iteration", file=sys.stderr, flush=True)
        n = int(xt)
        # algorithmic HBM bytes of the two Gram-Schmidt passes of iteration j
        # (16 B per complex element): dots read v_0..v_j and w, the update
        # reads w and v_0..v_j and writes w
        per_it = [2 * ((j + 2) + (j + 3)) * 16 * n for j in range(m - 1)]
        print(json.dumps({"krylov_probe": {"iterations": m, "theta_elems": n, "ms_per_iteration":
                                           1e3 * float(np.median(t_it[1:])),
                                           "gs_bytes_per_iteration_mean": float(np.mean(per_it))}}), flush=True)
        ctx.close()
        return

    heff_by_prec = {}
    ys = {}
    for name, p in (("fp64", T.FP64), ("fp32", T.FP32), ("bf16x3", T.BF16X3)):
        d, ys[name] = time_applies(p)
        heff_by_prec[name] = {"ms_per_apply": 1e3 * float(np.mean(d)), "ms_median": 1e3 * float(np.median(d)),
                              "ms_min": 1e3 * float(d.min()),
                              "tflops": flops / float(np.mean(d)) / 1e12}
        print(f"bench: H_eff apply {name} {heff_by_prec[name]['ms_per_apply']:.3f} ms, "
              f"{heff_by_prec[name]['tflops']:.2f} TFLOP/s", file=sys.stderr, flush=True)
    # the all-64x64 FP64 tiles on the hardware dispatcher's grid (one workgroup
    # per tile) and in the persistent launch (resident grid, device work
    # counter), and the all-32x32 tiles as wave tiles (four per workgroup)
    for mode, key in ((2, "fp64_dispatcher_grid"), (3, "fp64_persistent_grid"), (4, "fp64_wave_tiles")):
        before = os.environ.get("TDVP_FORCE_TILING")
        os.environ["TDVP_FORCE_TILING"] = str(mode)
        try:
            d, _ = time_applies(T.FP64)
        finally:
            restore_env("TDVP_FORCE_TILING", before)
        heff_by_prec["fp64"][key] = {"ms_per_apply": 1e3 * float(np.mean(d)), "tflops": flops / float(np.mean(d)) / 1e12}
        print(f"bench: H_eff apply FP64 tiling mode {mode}, {key}: {1e3 * float(np.mean(d)):.3f} ms", file=sys.stderr,
              flush=True)
    # the FP64 kernel the autotuner runs: the wave tiles when they are the faster
    # candidate (both forced timings above are of the same program)
    f64 = heff_by_prec["fp64"]
    fp64_kernel = ("heff_gemm_wave" if f64["fp64_wave_tiles"]["ms_per_apply"] < f64["fp64_dispatcher_grid"]["ms_per_apply"]
                   else "heff_gemm<double, 2, 2>")
    ctx.set_precision(prec)
    t_apply = heff_by_prec[args.prec]["ms_per_apply"] * 1e-3
    heff_tflops = heff_by_prec[args.prec]["tflops"]
    ref64 = ys["fp64"]
    for name in heff_by_prec:
        heff_by_prec[name]["rel_err_vs_fp64"] = float(np.linalg.norm(ys[name] - ref64) / np.linalg.norm(ref64))

    # ---- larger, more uneven blocks: chi = 16384 with log-normal sector dimensions,
    # grouped launch against one launch per output block ------------------------------
    # (each on a context of its own, closed afterwards, so that the sweeps below
    # start from the state a sweep-only run has: with the chi ~ 62 000 apply
    # and bond update run on the sweep's context, its splits took ~15 % longer)
    large = None
    if not args.no_large:
        lctx = T.Context(0, stream=stream.cuda_stream, precision=prec)
        large = large_heff(args, T, torch, stream, lctx, model)
        lctx.close()
    late = None
    if not args.no_late:
        lctx = T.Context(0, stream=stream.cuda_stream, precision=prec)
        late = large_heff(args, T, torch, stream, lctx, model, late=True)
        lctx.close()
        torch.cuda.empty_cache()
    abelian = None
    if not args.no_abelian:
        abelian = u1_heff(args, T, torch, stream, ctx, model, chi)
        abelian["su2_over_u1_time"] = heff_by_prec["fp64"]["ms_per_apply"] / abelian["fp64"]["ms_per_apply"]

    # ---- full sweeps: the step at the working precision, and the mixed path
    # (FP32 block products, FP64 Lanczos / SVD) from the same initial state ----
    sweep = {}
    mixed = None
    if args.steps > 0 or args.warmup > 0:
        bonds_r, sites_r = synth.random_mps(L, chi, args.seed + 100, center=1)
        Tr = [T.Bond(b) for b in bonds_r]

        def new_mps(c):
            bufs, descs = [], []
            for k in range(1, L + 1):
                tk, to, tt, _ = T.center_layout(Tr[k - 1], Tr[k], 1)
                d = dev(pack(sites_r[k - 1], tk, to, tt))
                bufs.append(d)
                descs.append(T.Blocks(tk, to, d.data_ptr(), tt))
            m = T.MPS.from_blocks(c, model, Tr, descs)
            torch.cuda.synchronize()
            return m

        run = dict(dt=0.05, eps_tol=1e-4, chi_cap=chi, krylov_tol=1e-10, krylov_maxdim=40)
        mps = new_mps(ctx)
        # the other precision rungs, each from the same initial state on its own context
        others = []
        if not args.no_mixed:
            rungs = [("fp32", T.FP32), ("bf16x3", T.BF16X3)] if prec == T.FP64 else [("fp64", T.FP64)]
            for name, p_ in rungs:
                octx = T.Context(0, stream=stream.cuda_stream, precision=p_)
                others.append({"name": name, "ctx": octx, "mps": new_mps(octx), "infos": [], "cmp": []})
            if prec == T.FP64:
                # the memory plan for the largest bonds on the benchmark's bond: inactive
                # tensors and environments in host memory, complex64 Krylov basis
                octx = T.Context(0, stream=stream.cuda_stream, precision=T.FP64)
                octx.set_host_staging(True)
                octx.set_krylov_storage(T.FP32)
                others.append({"name": "fp64_host_staged_complex64_krylov", "ctx": octx, "mps": new_mps(octx),
                               "infos": [], "cmp": []})
            for o in others:
                o["ctx"].memory(reset_peak=True)
        ctx.memory(reset_peak=True)
        infos = []
        t_sw = 0.0
        for st in range(args.warmup + args.steps):
            timed = st >= args.warmup
            ctx.synchronize()
            torch.cuda.synchronize()
            t0 = time.time()
            info = mps.sweep(run["dt"], eps_tol=run["eps_tol"], chi_cap=run["chi_cap"],
                             krylov_tol=run["krylov_tol"], krylov_maxdim=run["krylov_maxdim"])
            ctx.synchronize()
            torch.cuda.synchronize()
            if timed:
                t_sw += time.time() - t0
                infos.append(info)
            print(f"bench: {'timed' if timed else 'warmup'} sweep {st + 1}: {info['seconds']:.2f} s",
                  file=sys.stderr, flush=True)
            for o in others:
                other = o["mps"]
                oinfo = other.sweep(run["dt"], eps_tol=run["eps_tol"], chi_cap=run["chi_cap"],
                                    krylov_tol=run["krylov_tol"], krylov_maxdim=run["krylov_maxdim"])
                o["infos"].append(oinfo)
                ov = mps.overlap(other)
                n1, n2 = mps.overlap(mps).real, other.overlap(other).real
                sz1, dc1, _ = mps.measure()
                sz2, dc2, _ = other.measure()
                o["cmp"].append({"state_err": float(np.sqrt(max(n1 + n2 - 2 * ov.real, 0.0))),
                                 "d_sz": float(np.abs(sz1 - sz2).max()), "d_docc": float(np.abs(dc1 - dc2).max())})
                print(f"bench: {o['name']} sweep {st + 1}: {oinfo['seconds']:.2f} s, |psi-phi| "
                      f"{o['cmp'][-1]['state_err']:.2e}, max|dSz| {o['cmp'][-1]['d_sz']:.2e}",
                      file=sys.stderr, flush=True)
        sweep_peak = ctx.memory()[1]
        # one-site sweeps on the saturated state (bond dimensions fixed)
        one = []
        for st in range(args.one_site_steps):
            ctx.synchronize()
            info1 = mps.sweep1(run["dt"], krylov_tol=run["krylov_tol"], krylov_maxdim=run["krylov_maxdim"])
            one.append(info1)
            print(f"bench: one-site sweep {st + 1}: {info1['seconds']:.2f} s", file=sys.stderr, flush=True)
        if args.steps > 0:
            sweep = {
                "s_per_sweep": t_sw / args.steps,
                "sweep_heff_flops": float(np.mean([i["heff_flops"] for i in infos])),
                "sweep_env_flops": float(np.mean([i["env_flops"] for i in infos])),
                "sweep_phase_s": {k: float(np.mean([i[k] for i in infos])) for k in
                                  ("t_lanczos", "t_svd", "t_env")},
                "krylov_iters_per_sweep": float(np.mean([i["krylov_iters"] for i in infos])),
                "graph_replayed_iters_per_sweep": float(np.mean([i["graph_iters"] for i in infos])),
                "eig_fallbacks": int(sum(i["eig_fallbacks"] for i in infos)),
                "max_chi": int(max(i["max_chi"] for i in infos)),
                "max_discarded": float(max(i["max_discarded"] for i in infos)),
                "peak_device_gb": sweep_peak / 1e9,
                "split_eigensolver": {
                    "in_house_reduction_from": os.environ.get("TDVP_EIG_TRD_MIN", "256"),
                    "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES", ""),
                    "note": "Gram matrices of buckets >= in_house_reduction_from: in-house Householder reduction "
                            "(one launch per column for all of a split's matrices), library tridiagonal divide "
                            "and conquer, in-house back-transformation; smaller ones: library batched solver"},
            }
            if one:
                sweep["one_site"] = {
                    "s_per_sweep": float(np.mean([i["seconds"] for i in one])),
                    "sweep_phase_s": {k: float(np.mean([i[k] for i in one])) for k in
                                      ("t_lanczos", "t_svd", "t_env")},
                    "krylov_iters_per_sweep": float(np.mean([i["krylov_iters"] for i in one])),
                    "note": "one-site TDVP sweeps continuing from the saturated two-site state "
                            "(QR gauge moves instead of SVD splits; bond dimensions fixed)"}
        for o in others:
            tail = o["infos"][args.warmup:] or o["infos"]
            cmp = o["cmp"]
            rec = {
                "precision": o["name"],
                "peak_device_gb": o["ctx"].memory()[1] / 1e9,
                "s_per_sweep": float(np.mean([i["seconds"] for i in tail])),
                "sweep_phase_s": {k: float(np.mean([i[k] for i in tail])) for k in
                                  ("t_lanczos", "t_svd", "t_env")},
                "state_err_first_step": cmp[0]["state_err"],
                "state_err_after_all": cmp[-1]["state_err"],
                "max_obs_err": max(max(c["d_sz"], c["d_docc"]) for c in cmp),
                "sweeps_compared": len(cmp),
                "note": "both runs start from the same seeded random MPS; errors are |psi_ref - psi_rung| and "
                        "max over sites of |d<S^z>|, |d<n_up n_dn>| after each sweep",
            }
            if mixed is None:
                mixed = rec
            else:
                mixed.setdefault("other_rungs", []).append(rec)
            o["mps"].close()
            o["ctx"].close()
        mps.close()

    abelian_sweep = None
    if not args.no_abelian and (args.steps > 0 or args.warmup > 0):
        abelian_sweep = u1_sweep(args, T, torch, stream, ctx, model, chi,
                                 dict(dt=0.05, eps_tol=1e-4, chi_cap=chi, krylov_tol=1e-10, krylov_maxdim=40))

    # ---- CPU baseline: the oracle on sampled output blocks ------------------------
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import sampled as S
        try:
            from threadpoolctl import threadpool_info
            cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
        except Exception:
            cores = len(os.sched_getaffinity(0))
        Lkeys = [tuple(int(v) for v in k) for k in Ld[0]]
        Rkeys = [tuple(int(v) for v in k) for k in Rd[0]]
        # environment block values for the oracle come from the same seeded generator
        # path as the GPU ones only through the GPU env chain, which the oracle may not
        # read; the oracle gets its own synthetic environments for the sampled blocks
        Lsyn = synth.block_data(Lkeys, [(bonds[site - 1][k[0]][2], bonds[site - 1][k[2]][2]) for k in Lkeys],
                                args.seed + 2, 11)
        Rsyn = synth.block_data(Rkeys, [(bonds[site + 1][k[0]][2], bonds[site + 1][k[2]][2]) for k in Rkeys],
                                args.seed + 3, 12)
        out_flops = {}
        for kind, out, inn, env, coef in terms:
            k = tuple(int(v) for v in xk[out])
            if kind == 0:
                f = 8.0 * bonds[site - 1][Lkeys[env][0]][2] * xd[inn][0] * xd[inn][1]
            elif kind == 1:
                f = 8.0 * xd[inn][0] * xd[inn][1] * bonds[site + 1][Rkeys[env][0]][2]
            else:
                f = 0.0
            out_flops[k] = out_flops.get(k, 0.0) + f
        cand = sorted(out_flops, key=lambda k: np.prod(S.restricted_dims(bonds[site - 1], bonds[site + 1],
                                                                         Lkeys, Rkeys, k)))
        cand = cand[len(cand) // 3:]
        rng = np.random.default_rng(0)
        rng.shuffle(cand)
        done_f, n_blocks, t0 = 0.0, 0, time.time()
        for k in cand:
            S.heff2_block(bonds[site - 1], bonds[site + 1], Lsyn, Rsyn, xs, k, site, t_h, U)
            done_f += out_flops[k]
            n_blocks += 1
            if time.time() - t0 > args.cpu_seconds:
                break
        t_cpu = time.time() - t0
        cpu = {"value": done_f / t_cpu / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"{n_blocks} output blocks of the chi=4096 middle-bond H_eff apply, each evaluated by "
                         f"the dense oracle on the sector-restricted expanded problem ({t_cpu:.1f} s); rate = "
                         f"algorithmic flops of those blocks / oracle time"}

    line = {
        "metric": METRIC,
        "value": heff_tflops,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sweep["s_per_sweep"] if "s_per_sweep" in sweep else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == T.FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"L={L} U(1)xSU(2) Hubbard (t=1, U=4) random MPS, chi={chi} full-state units, "
                               "Table-S2-shaped sectors; H_eff.Theta at sites 30-31 + full two-site TDVP sweep "
                               "(dt=0.05, eps_tol=1e-4, chi cap)",
                   "L": L, "chi": chi, "precision": args.prec},
        "heff": {"flops_per_apply": flops, "ms_per_apply": 1e3 * t_apply,
                 "blocks": len(xk), "terms": len(terms), "theta_elems": int(xt),
                 "env_chain_s": t_env_chain, "by_precision": heff_by_prec,
                 "roofline_by_precision": rooflines(heff_by_prec)},
        "roofline": {"bound": "mfma", "achieved": heff_tflops, "peak": PEAK[args.prec], "unit": "TFLOP/s",
                     "frac": heff_tflops / PEAK[args.prec], "traffic": measured_traffic(args.prec),
                     "kernel": fp64_kernel if prec == T.FP64 else "heff_gemm<float, 2, 2>"},
        "cpu_baseline": cpu,
        "mixed": mixed,
        "large_blocks": large,
        "late_time_blocks": late,
        "u1xu1_heff": abelian,
        "u1xu1_sweep": abelian_sweep,
    }
    line.update(sweep)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
