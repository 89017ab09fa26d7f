"""Benchmark of the even-odd Wilson operator on one MI355X.

One step = one application of M = 1 - kappa^2 H_eo H_oe to a 32^3x64 even
spinor (kappa = 0.126, links exp(0.5 i H), Gaussian source), i.e. the two hop
kernels of the operator.  ``value`` is 1320 * V flop per step over the timed
steps (GFlop/s), with every input resident in HBM before timing starts.

The JSON line also carries:
  gflops_1368   the same rate under the 1368 flop/site count (the 1320 count
                plus the 48 flop of the diagonal a*x+y on 12 complex numbers);
  roofline      the dominant kernel (the hop) against the 8 TB/s HBM peak, its
                average duration measured here with HIP events on the stream it
                runs on, its fraction of a measured 1 GiB device copy, and
                L2-to-memory traffic from the committed rocprofv3 counters when
                they were taken on the current kernel source;
  cpu_baseline  the FP64 NumPy oracle timed on a sample of the same workload
                on this host (single thread; CPU model and count stated), and
                its apply time at 4^4 and 16^3x32;
  variants      the same apply in other storage formats;
  clover        the even-odd operator with site-local D_ee, D_oo blocks (FP32/18
                and FP16/12) and its mixed-precision solve;
  t_split_32x32x32x8, grid_2x2x2x2_block_32x32x32x64
                one device's share of 32^3x64 cut along t into 8 slabs, and of
                64^3x128 on a 2^4 grid: the block hop as bulk kernel + face
                pack + face unpack (faces exchanged with itself) against the
                block's periodic hop, eager and captured as a HIP graph;
  solve         solve times to a true FP64 residual of 1e-10 (and FP32 CGLS to
                1e-6): FP64 defect correction with FP16/BF16 inner solves
                against FP32 inner solves, for one source at 32^3x64, twelve
                point+noise sources at 32^3x64 (batched vs one at a time) and
                one source at 48^3x96.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--format f32/f32/18]
                    [--no-solve] [--no-cpu] [--profile-mode | --profile-solve | --profile-split |
                     --profile-shapes]
"""
from __future__ import annotations

import os

# the oracle baseline is single-threaded; keep BLAS from spawning threads
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import argparse
import hashlib
import json
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DIMS = (32, 32, 32, 64)
KAPPA = 0.126
EPS = 0.5
SEED_GAUGE, SEED_SRC = 201, 202
FLOP_SITE = 1320
REAL = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}


# Launch shapes of --profile-shapes (weo_set_mrhs_shape arguments): the packed
# FP16 link-resident kernel in several workgroup sizes and schedules (z strips
# of 2, 4, 8 planes, half-plane columns of 4, 8, 16), the LDS-staged kernel,
# and one lane per (site, rhs).
PROFILE_SHAPES = [(-4, 256, 0, 8, 0), (-4, 256, 0, 4, 0), (-4, 256, 0, 0, 0), (-4, 64, 0, 8, 0), (-4, 64, 1, 8, 0),
                  (-4, 256, 1, 2, 0), (-4, 256, 0, -4, 0), (-4, 256, 0, -8, 0), (-4, 256, 0, -16, 0),
                  (-2, 256, 0, 8, 0), (-5, 2, 0, 4, 0), (-5, 8, 0, 4, 0), (1, 0, 0, 0, 0)]


def hop_bytes_per_site(sp, lp, reals):
    """Algorithmic bytes of one hop per output site: 8 links, one input and one
    output spinor record (each field touched once)."""
    return 8 * reals * REAL[lp] + 2 * 24 * REAL[sp]


def apply_bytes_per_site(sp, lp, reals):
    """Per full-lattice site of one M apply: two hops over V/2 sites each and
    the even input read once more for the axpy."""
    return hop_bytes_per_site(sp, lp, reals) + 12 * REAL[sp]


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2303_08609_amd", "csrc")
    for f in ("hop.hip", "hop_core.h", "weo_device.h", "weo_geom.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(fmt_key):
    """HBM bytes per hop launch from profiles/hop_traffic.json, if those
    counters were taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "hop_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    e = d.get("formats", {}).get(fmt_key)
    if not e or d.get("kernel_source_sha") != kernel_source_hash():
        return None
    return e.get("hbm_bytes_per_launch")


def cpu_baseline(budget_s=15.0):
    """FP64 oracle M apply on a 32^3x8 slab (1/8 of the workload volume, same
    per-site work), repeated until ``budget_s`` seconds are used; plus the
    oracle's apply time (median of three) on the 4^4 and 16^3x32 lattices of
    the smaller workloads.  One thread (BLAS threads pinned to 1)."""
    from oracle import wilson as W
    from paper_2303_08609_amd import inputs
    ph = np.array([1, 1, 1, -1], dtype=np.complex128)
    dims = (32, 32, 32, 8)
    u = inputs.gen_gauge(dims, EPS, SEED_GAUGE)
    psi = inputs.gen_spinor_half(dims, SEED_SRC)
    v = 32 * 32 * 32 * 8
    n, t0 = 0, time.perf_counter()
    while True:
        W.apply_m(u, psi, KAPPA, ph)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s or n >= 10:
            break
    sizes = {}
    for d, kappa, eps in (((4, 4, 4, 4), 0.125, 0.3), ((16, 16, 16, 32), 0.125, 0.5)):
        us = inputs.gen_gauge(d, eps, 11)
        ps = inputs.gen_spinor_half(d, 12)
        runs = []
        for _ in range(3):
            t1 = time.perf_counter()
            W.apply_m(us, ps, kappa, ph)
            runs.append(time.perf_counter() - t1)
        vs = d[0] * d[1] * d[2] * d[3]
        med = sorted(runs)[1]
        sizes["x".join(map(str, d))] = {"apply_seconds": round(med, 5),
                                        "gflops": round(FLOP_SITE * vs / med / 1e9, 4)}
    return {"value": round(FLOP_SITE * v * n / dt / 1e9, 4), "unit": "GFlop/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n} oracle M applies on a 32^3x8 slab (1/8 of 32^3x64), FP64 NumPy, "
                      f"{dt:.1f} s",
            "host_cpu": host_cpu(),
            "oracle_apply_at": sizes}


def split_timings(blat, dirs, ud, xd, fmt, n, warmup, time_loop):
    """One device's share of a hop split along ``dirs``: the block's hop with
    those directions open (bulk), the faces packed in each open direction and
    added back after a self-exchange (periodic wrap: the block is its own
    neighbour), in microseconds per hop; eager launches, the face pack on a
    second stream, and the whole sequence captured as one HIP graph (both
    orders).  Every graph replay is checked bit for bit against the eager
    result first."""
    import torch
    bopen = blat.open_dirs(dirs)
    out = blat.new_spinor(fmt)
    bufs = {mu: blat.face_pack(ud, xd, fmt, 1, mu=mu) for mu in dirs}

    def pack():
        for mu in dirs:
            blat.face_pack(ud, xd, fmt, 1, lo=bufs[mu][0], hi=bufs[mu][1], mu=mu)

    def unpack():
        for mu in dirs:
            ph = blat.bc[mu]
            blat.face_unpack(ud, bufs[mu][1], bufs[mu][0], out, fmt, 1, phase_lo=ph, phase_hi=ph, mu=mu)

    plain = lambda: blat.hop(ud, xd, fmt, 1, out=out)
    bulk = lambda: bopen.hop(ud, xd, fmt, 1, out=out)
    side = torch.cuda.Stream()          # default priority

    def whole():
        pack()
        bulk()
        unpack()

    def overlapped():
        # faces packed on a second stream while the bulk kernel runs, as a
        # sharded hop posts them before its interior work
        cur = torch.cuda.current_stream()
        side.wait_stream(cur)
        with torch.cuda.stream(side):
            pack()
        bulk()
        cur.wait_stream(side)
        unpack()

    plain()
    want = blat.unpack_spinor(out, fmt)
    whole()
    torch.cuda.synchronize()
    ref = out.clone()
    # the faces are added after the bulk sum: equal to the periodic hop up
    # to the storage format's rounding
    err = (torch.linalg.vector_norm(blat.unpack_spinor(ref, fmt) - want) / torch.linalg.vector_norm(want)).item()
    if err > {"f64": 1e-12, "f32": 1e-6}.get(fmt.spinor, 2e-2):
        raise RuntimeError(f"split hop over {dirs} differs from the periodic hop by {err:.2e}")
    graphs = {}
    for name, fn in (("graph_pack_bulk_unpack_us", whole), ("graph_overlapped_us", overlapped)):
        fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        for _ in range(3):
            out.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            if not torch.equal(out, ref):
                raise RuntimeError(f"graph replay of the split hop over {dirs} differs")
        graphs[name] = g
    r = {}
    for name, fn in (("periodic_hop_us", plain), ("bulk_hop_us", bulk), ("face_pack_us", pack),
                     ("face_unpack_us", unpack), ("pack_bulk_unpack_us", whole),
                     ("pack_overlapped_bulk_unpack_us", overlapped),
                     ("graph_pack_bulk_unpack_us", graphs["graph_pack_bulk_unpack_us"].replay),
                     ("graph_overlapped_us", graphs["graph_overlapped_us"].replay)):
        for _ in range(warmup):
            fn()
        r[name] = round(time_loop(fn, n) * 1e3, 2)
    r["face_bytes_each_direction"] = {str(mu): blat.face_bytes(fmt, mu=mu) for mu in dirs}
    del graphs
    return r


def copy_gbs(time_loop, nbytes=1 << 30):
    """Read+write bandwidth of a plain device copy of ``nbytes`` (the torch
    D2D copy and a float4-wide elementwise kernel; the faster one is the
    practical ceiling a streaming kernel can reach)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    res = {}
    for name, fn in (("memcpy", lambda: dst.copy_(src)),
                     ("elementwise", lambda: torch.mul(src, 1.0, out=dst))):
        for _ in range(3):
            fn()
        ms = time_loop(fn, 20)
        res[name] = round(2 * nbytes / (ms * 1e-3) / 1e9, 1)
    del src, dst
    torch.cuda.empty_cache()
    return res


def host_cpu():
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def parse_fmt(s):
    sp, lp, reals = s.split("/")
    return sp, lp, int(reals)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--format", default="f32/f32/18")
    ap.add_argument("--variants", default="f32/f32/12,f64/f64/18,f16/f16/12,bf16/f16/12")
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the solver timings (32^3x64 single and 12 rhs, 48^3x96)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-solve", action="store_true",
                    help="short fixed run for rocprofv3: the 12-source 32^3x64 solve to 1e-10 "
                         "(FP64 defect correction around --solve-inner / --solve-method inner "
                         "solves), once to tune, once more")
    ap.add_argument("--solve-inner", default="f16/f16/12", help="inner format of --profile-solve")
    ap.add_argument("--solve-method", default="bicgstab", choices=["cg", "bicgstab", "blockcg"],
                    help="inner method of --profile-solve")
    ap.add_argument("--profile-split", action="store_true",
                    help="short fixed run for rocprofv3: one device's share of the t-split hop at "
                         "32^3x8, sequential and with the face pack on a second stream, --steps each")
    ap.add_argument("--profile-shapes", action="store_true",
                    help="short fixed run for rocprofv3 --pmc: the FP16/12 multi-rhs hop at 32^3x64 in "
                         "fixed launch shapes for 12, 6 and 3 right-hand sides, 3 launches each")
    ap.add_argument("--profile-mode", action="store_true",
                    help="short fixed run for rocprofv3: a 1 GiB device copy (counter "
                         "calibration) and --steps hop launches per format, nothing else")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU "
              "decomposition is a design, not a built path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2303_08609_amd import inputs
    from paper_2303_08609_amd.ops import Format, Lattice, to_device

    torch.cuda.set_device(0)
    if a.profile_solve:
        from paper_2303_08609_amd.solve import F64_OUTER, cg
        lat12 = Lattice(DIMS, KAPPA, (1, 1, 1, -1))
        ud = to_device(inputs.gen_gauge(DIMS, EPS, 401))
        f64, fi = Format(*F64_OUTER), Format(*parse_fmt(a.solve_inner))
        u64, ui = lat12.pack_gauge(ud, f64), lat12.pack_gauge(ud, fi)
        b12 = lat12.pack_spinor(to_device(inputs.gen_point_noise_sources(DIMS, 406)), f64)
        for k in range(2):
            x, info = cg(lat12, f64, u64, b12, nrhs=12, tol=1e-10, inner=fi, u_inner=ui,
                         inner_tol=1e-5 if a.solve_inner.startswith("f32") else 1e-3,
                         maxiter=50000, max_outer=100, method=a.solve_method)
            torch.cuda.synchronize()
            print(f"[bench] profiled 12-rhs solve {k}: {info['seconds']:.4f} s, inner {info['iters']}, "
                  f"outer {info['outer_iters']}", file=sys.stderr, flush=True)
        return
    if a.profile_shapes:
        from paper_2303_08609_amd import wilson_eo as WE
        lat12 = Lattice(DIMS, KAPPA, (1, 1, 1, -1))
        f2 = Format("f16", "f16", 12)
        ud = lat12.pack_gauge(to_device(inputs.gen_gauge(DIMS, EPS, 401)), f2)
        xd = lat12.pack_spinor(to_device(inputs.gen_point_noise_sources(DIMS, 406)), f2)
        out = lat12.new_spinor(f2, 12)
        for sh in PROFILE_SHAPES:
            WE.check(WE.weo_set_mrhs_shape(*sh), "weo_set_mrhs_shape")
            for nr in (12, 6, 3):
                for _ in range(3):
                    lat12.hop(ud, xd, f2, out_parity=1, nrhs=nr, out=out)
                torch.cuda.synchronize()
                print(f"[bench] profiled shape {sh}, {nr} rhs", file=sys.stderr, flush=True)
        WE.weo_set_mrhs_shape(0, 0, 0, 0, 0)
        return
    if a.profile_split:
        sdims = (32, 32, 32, 8)
        slat = Lattice(sdims, KAPPA, (1, 1, 1, -1))
        sopen = slat.open_t()
        f2 = Format("f32", "f32", 18)
        ud = slat.pack_gauge(to_device(inputs.gen_gauge(sdims, EPS, SEED_GAUGE)), f2)
        xd = slat.pack_spinor(to_device(inputs.gen_spinor_half(sdims, SEED_SRC)), f2)
        out = slat.new_spinor(f2)
        lo, hi = slat.face_pack(ud, xd, f2, 1)
        stream = torch.cuda.current_stream()
        side = torch.cuda.Stream()
        for mode in ("sequential", "overlapped"):
            for _ in range(a.steps):
                if mode == "sequential":
                    slat.face_pack(ud, xd, f2, 1, lo=lo, hi=hi)
                    sopen.hop(ud, xd, f2, 1, out=out)
                else:
                    side.wait_stream(stream)
                    with torch.cuda.stream(side):
                        slat.face_pack(ud, xd, f2, 1, lo=lo, hi=hi)
                    sopen.hop(ud, xd, f2, 1, out=out)
                    stream.wait_stream(side)
                slat.face_unpack(ud, hi, lo, out, f2, 1, phase_lo=-1.0, phase_hi=-1.0)
            torch.cuda.synchronize()
            print(f"[bench] profiled {a.steps} t-split hops ({mode})", file=sys.stderr, flush=True)
        return
    lat = Lattice(DIMS, KAPPA, (1, 1, 1, -1))
    v = lat.volume
    t0 = time.perf_counter()
    u = inputs.gen_gauge(DIMS, EPS, SEED_GAUGE)
    psi = inputs.gen_spinor_half(DIMS, SEED_SRC)
    print(f"[bench] inputs generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    u_dev64 = to_device(u)
    psi_dev64 = to_device(psi)
    stream = torch.cuda.current_stream()

    def time_loop(fn, n):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n          # ms

    def run_format(fs, steps, warmup):
        fmt = Format(*fs)
        ud = lat.pack_gauge(u_dev64, fmt)
        xd = lat.pack_spinor(psi_dev64, fmt)
        out = lat.new_spinor(fmt)
        tmp = lat.new_spinor(fmt)
        apply = lambda: lat.apply(ud, xd, fmt, out=out, tmp=tmp)
        hop = lambda: lat.hop(ud, xd, fmt, out_parity=1, out=tmp)
        for _ in range(warmup):
            apply()
        ms_apply = time_loop(apply, steps)
        for _ in range(warmup):
            hop()
        ms_hop = time_loop(hop, max(steps, 1))
        del ud, xd, out, tmp
        return ms_apply, ms_hop

    if a.profile_mode:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        for _ in range(5):
            dst.copy_(src)
        del src, dst
        for vs in [a.format] + [s for s in a.variants.split(",") if s]:
            f2 = Format(*parse_fmt(vs))
            ud = lat.pack_gauge(u_dev64, f2)
            xd = lat.pack_spinor(psi_dev64, f2)
            tmp = lat.new_spinor(f2)
            for _ in range(a.steps):
                lat.hop(ud, xd, f2, out_parity=1, out=tmp)
            torch.cuda.synchronize()
            print(f"[bench] profiled {a.steps} hop launches of {vs}", file=sys.stderr, flush=True)
            del ud, xd, tmp
        # twelve right-hand sides through the multi-rhs kernel (tuned shape)
        b12 = torch.from_numpy(inputs.gen_point_noise_sources(DIMS, 406)).cuda()
        for vs in ("f32/f32/18", "f16/f16/12", "f64/f64/12"):
            f2 = Format(*parse_fmt(vs))
            ud = lat.pack_gauge(u_dev64, f2)
            xd = lat.pack_spinor(b12, f2)
            tmp = lat.new_spinor(f2, 12)
            lat.hop(ud, xd, f2, out_parity=1, nrhs=12, out=tmp)         # tunes the shape
            for _ in range(a.steps):
                lat.hop(ud, xd, f2, out_parity=1, nrhs=12, out=tmp)
            torch.cuda.synchronize()
            print(f"[bench] profiled {a.steps} 12-rhs hop launches of {vs}", file=sys.stderr, flush=True)
            del ud, xd, tmp
        return

    fs = parse_fmt(a.format)
    ms_apply, ms_hop = run_format(fs, a.steps, a.warmup)
    print(f"[bench] {a.format}: apply {ms_apply * 1e3:.1f} us, hop {ms_hop * 1e3:.1f} us",
          file=sys.stderr, flush=True)
    gflops = FLOP_SITE * v / (ms_apply * 1e-3) / 1e9
    hop_bytes = hop_bytes_per_site(*fs) * (v // 2)
    achieved = hop_bytes / (ms_hop * 1e-3) / 1e9
    fmt_key = "/".join(map(str, fs))
    traffic = traffic_from_profiles(fmt_key)
    copy = copy_gbs(time_loop)
    copy_best = max(copy.values())
    print(f"[bench] device copy GB/s: {copy}", file=sys.stderr, flush=True)

    variants = {}
    for vs in [s for s in a.variants.split(",") if s]:
        f2 = parse_fmt(vs)
        m_a, m_h = run_format(f2, max(a.steps // 4, 1), a.warmup)
        variants[vs] = {
            "us_per_apply": round(m_a * 1e3, 2),
            "gflops": round(FLOP_SITE * v / (m_a * 1e-3) / 1e9, 1),
            "apply_gbs": round(apply_bytes_per_site(*f2) * v / (m_a * 1e-3) / 1e9, 1),
            "hop_us": round(m_h * 1e3, 2),
            "hop_frac_hbm": round(hop_bytes_per_site(*f2) * (v // 2) / (m_h * 1e-3) / 1e9
                                  / HBM_PEAK_GBS, 4),
        }
        print(f"[bench] {vs}: {variants[vs]}", file=sys.stderr, flush=True)

    # one device's share of a t-split 32^3x64 lattice over 8 devices (a
    # 32^3x8 slab, t open) and of 64^3x128 over a 2^4 grid (a 32^3x64 block,
    # every direction open): bulk hop + face pack + face unpack with the
    # faces exchanged with itself, against the block's periodic hop; eager
    # and as one captured HIP graph
    split = {}
    sdims = (32, 32, 32, 8)
    slat = Lattice(sdims, KAPPA, (1, 1, 1, -1))
    su = to_device(inputs.gen_gauge(sdims, EPS, SEED_GAUGE))
    spsi = to_device(inputs.gen_spinor_half(sdims, SEED_SRC))
    for vs in ("f32/f32/18", "f16/f16/12"):
        f2 = Format(*parse_fmt(vs))
        ud = slat.pack_gauge(su, f2)
        xd = slat.pack_spinor(spsi, f2)
        split[vs] = split_timings(slat, (3,), ud, xd, f2, max(a.steps // 4, 1), a.warmup, time_loop)
        print(f"[bench] t-split 32^3x8 {vs}: {split[vs]}", file=sys.stderr, flush=True)
        del ud, xd
    del su, spsi
    grid4 = {}
    for vs in ("f32/f32/18", "f16/f16/12"):
        f2 = Format(*parse_fmt(vs))
        ud = lat.pack_gauge(u_dev64, f2)
        xd = lat.pack_spinor(psi_dev64, f2)
        grid4[vs] = split_timings(lat, (0, 1, 2, 3), ud, xd, f2, max(a.steps // 4, 1), a.warmup, time_loop)
        print(f"[bench] 2^4 grid, 32^3x64 block {vs}: {grid4[vs]}", file=sys.stderr, flush=True)
        del ud, xd

    # clover-type operator (site-local D_ee, D_oo): the same lattice with
    # random Hermitian site blocks near 1, packed as inverses
    clover = {}
    blocks = to_device(inputs.gen_site_blocks(DIMS, 0.3, 207))
    for vs in ("f32/f32/18", "f16/f16/12"):
        sp_, lp_, re_ = parse_fmt(vs)
        f2 = Format(sp_, lp_, re_)
        ud = lat.pack_gauge(u_dev64, f2)
        xd = lat.pack_spinor(psi_dev64, f2)
        clv = lat.pack_clover(blocks, f2)
        out = lat.new_spinor(f2)
        tmp = lat.new_spinor(f2)
        fn = lambda: lat.clover_apply(ud, clv, xd, f2, out=out, tmp=tmp)
        for _ in range(a.warmup):
            fn()
        ms = time_loop(fn, max(a.steps // 4, 1))
        cb = 2 * 18 * 2 * REAL[lp_]                     # two blocks of 18 complex per site
        byts = (apply_bytes_per_site(sp_, lp_, re_) + cb) * v
        clover[vs] = {"us_per_apply": round(ms * 1e3, 2),
                      "gflops_1320": round(FLOP_SITE * v / (ms * 1e-3) / 1e9, 1),
                      "bytes_per_site": apply_bytes_per_site(sp_, lp_, re_) + cb,
                      "apply_gbs": round(byts / (ms * 1e-3) / 1e9, 1),
                      "frac_hbm": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        print(f"[bench] clover {vs}: {clover[vs]}", file=sys.stderr, flush=True)
        del ud, xd, clv, out, tmp
    if not a.no_solve:
        from paper_2303_08609_amd import solve as S
        clover["solve_1e-10"] = S.bench_clover_solve(lat, u_dev64, psi_dev64, blocks)
        print(f"[bench] clover solves: {clover['solve_1e-10']}", file=sys.stderr, flush=True)
    del blocks

    solve = None
    if not a.no_solve:
        from paper_2303_08609_amd import solve as S
        solve = {"32^3x64_single_rhs": S.bench_solves(lat, u, psi, u_dev64, psi_dev64)}
        print(f"[bench] single-rhs solves: {solve}", file=sys.stderr, flush=True)
        del u_dev64, psi_dev64
        torch.cuda.empty_cache()
        solve["32^3x64_12rhs_point_noise"] = S.bench_solves_12rhs()
        print(f"[bench] 12-rhs solves: {solve['32^3x64_12rhs_point_noise']}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        solve["48^3x96_mixed"] = S.bench_solves_large()
        print(f"[bench] 48^3x96 solves: {solve['48^3x96_mixed']}", file=sys.stderr, flush=True)

    line = {
        "metric": "eo-Wilson GFlop/s + % HBM roofline (32^3\u00d764); mixed vs FP32 solve time",
        "value": round(gflops, 1),
        "unit": "GFlop/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_apply, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fs[0] == "f32" else fs[0],
        "data": "synthetic: seeded near-unit SU(3) links exp(0.5 i H) and a Gaussian source",
        "config": {"workload": "even-odd Wilson M apply, 32^3x64, "
                               f"{fs[0]} spinors, {fs[1]} links with {fs[2]} reals",
                   "lattice": list(DIMS), "kappa": KAPPA, "link_eps": EPS,
                   "bc": "periodic x,y,z; antiperiodic t",
                   "flop_per_site": FLOP_SITE,
                   "apply_bytes_per_site": apply_bytes_per_site(*fs),
                   "apply_frac_hbm": round(apply_bytes_per_site(*fs) * v / (ms_apply * 1e-3) / 1e9
                                           / HBM_PEAK_GBS, 4)},
        "gflops_1368": round(gflops * 1368 / FLOP_SITE, 1),
        "roofline": {"bound": "hbm", "kernel": "k_hop (one hopping block, V/2 output sites)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_kind": "L2-to-memory bytes per launch (TCC FETCH_SIZE + WRITE_SIZE, "
                                     "scaled by a 1 GiB copy's reading); null when the kernel "
                                     "source changed since they were taken",
                     "hop_us": round(ms_hop * 1e3, 2),
                     "bytes_per_launch": hop_bytes,
                     "copy_gbs": copy,
                     "frac_of_copy": round(achieved / copy_best, 4)},
        "variants": variants,
        "t_split_32x32x32x8": split,
        "grid_2x2x2x2_block_32x32x32x64": grid4,
        "clover": clover,
    }
    if solve is not None:
        line["solve"] = solve
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
