#!/usr/bin/env python3
"""Throughput of the FSA likelihood + gradient step on one MI355X.

Workload (synthetic, seeded): n = 500,000 locations uniform on [0,1]^2,
Matérn-3/2 (sigma1^2 = 1, rho = 0.05, sigma^2 = 0.1), m = 500 inducing points
by kmeans++ on a 20k subsample, Wendland taper with ~80 nonzeros per row,
y from 2,000 random Fourier features plus noise, t = 50 Rademacher probes.

One step = the whole hot path from device-resident inputs: grid binning and
taper pattern, covariance generation and whitening, residual values,
FITC capacitance and its Cholesky factor, probes, block PCG with Lanczos
coefficients, SLQ log-determinant, and the stochastic gradient.
`value` = PCG probe-iterations executed per second of step time in the
mixed-precision mode (float32 blocks, float64 inner products, float64
residual replacement); the float64 run is reported beside it.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0}
KERNELS = ["sparse_product", "update_and_reduce", "woodbury_expand", "direction_update", "small"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# rocprofv3 kernel names of the four PCG kernel classes, per element type
KERNEL_NAMES = {
    "f32": ["k_spmm_tiled<2, 4>", "k_reduce_split<true, 1, 4>", "k_rows_split<2, 8, 4>", "k_pcg_hupdate<float, float>"],
    "f32mfma": ["k_spmm_tiled<2, 4>", "k_reduce_gemm_f32<float, true, 1>", "k_rows_gemm_f32<float, true, 2>",
                "k_pcg_hupdate<float, float>"],
    "bf16a": ["k_spmm_tiled<2, 4>", "k_reduce_bf16<true, 1>", "k_rows_bf16<2>", "k_pcg_hupdate<float, float>"],
    "f64": ["k_spmm_dense<double, 2>", "k_reduce_gemm_f64<true, 1>",
            "k_rows_gemm_f64<true, 2, 3>", "k_pcg_hupdate<double, double>"],
}
COUNTERS = os.path.join(ROOT, "profiles", "pcg_kernels_n500k_m500_t50_counters.md")


def kernel_work(k, n, m, tp, nnz, b, ba=None):
    """Algorithmic (bytes, flops) per launch of kernel class k with element
    size b (block vectors and sparse values) and ba (low-rank factor, b if
    None); the solution accumulates in float64 (float64 operator) or as
    float32 increments folded into float64 at each residual replacement.
    Every operand counted once."""
    blk = n * tp
    ba = b if ba is None else ba
    if k == 0:   # V = S H + P, h.v: key (4 B) + value per nonzero, H in, P in, V out, row pointers (the
        #          float32 product reads the same values as MFMA-order tiles, zeros included: the
        #          algorithmic figure stays that of the compressed rows)
        return nnz * (b + 4) + 8 * (n + 1) + 3 * blk * b, 2.0 * nnz * tp
    if k == 1:   # r -= a v (R in/out, V in), W = A D^-1 r: A (n x m) once, D^-1
        return n * m * ba + 3 * blk * b + 8 * n, 2.0 * n * m * tp
    if k == 2:   # t = A g, r.q with q = (r - t)/D: A once, R in, T out, D^-1
        return n * m * ba + 2 * blk * b + 8 * n, 2.0 * n * m * tp
    if k == 3:   # u += a h (U in/out: float64, or the float32 increment block with a float32 operator),
        #          h = (r - t)/D + beta h, p = t + beta p: R, T, H, P in; H, P out
        return blk * (6 * b + (8 if b == 4 else 16)) + 8 * n, 6.0 * blk
    return 0, 0


def _code_text(src):
    """C/C++ source without its comments, whitespace runs collapsed to one
    space (string and character literals kept as written)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_fingerprint():
    """sha256 over the code (comments and layout ignored) of the sources that
    define the PCG kernels the hardware counters measure (their code, launch
    shapes and the grid layout they read) and of the ABI header: traffic is
    reported only for the code it was measured on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2405_14492_amd", "csrc")
    paths = [os.path.join(csrc, f) for f in ("common.hpp", "gemm.hpp", "geom.hip", "kernels.hpp", "ops.hip")]
    paths.append(os.path.join(ROOT, "include", "fsa.h"))
    for path in paths:
        h.update(os.path.basename(path).encode())
        with open(path, encoding="utf-8") as fh:
            h.update(_code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel_name):
    """HBM bytes per launch (fetch + write, copy-calibrated) of a kernel from
    the committed counter summary, or None if absent or measured on other
    sources."""
    try:
        with open(COUNTERS) as fh:
            lines = [ln for ln in fh if ln.startswith("traffic-json: ")]
    except OSError:
        return None
    if not lines:
        return None
    rec = json.loads(lines[-1][len("traffic-json: "):])
    if rec.get("fingerprint") != source_fingerprint():
        return None
    k = rec.get("kernels", {}).get(kernel_name)
    if not k:
        return None
    return k["fetch_bytes"] + k["write_bytes"]


def run_mode(F, dev, w, precision, steps, warmup, tol, torch, rr_period=20, fp32_products=0):
    """Warmup, then one untimed step with every kernel class timed by HIP
    events (per-class launch averages; the dominant class), then the timed
    steps with only the dominant class timed (each timed launch adds two event
    records to the stream, about 3 us each)."""
    def options(profile):
        return F.make_options(num_probes=w.num_probes, seed=w.seed, tol=tol, max_iter=1000, precision=precision,
                              rr_period=rr_period, profile=profile, fp32_products=fp32_products)
    theta = w.theta

    def step(opt):
        ctx = F.fsa_build_dev(dev["locs"], dev["y"], theta, dev["ind"], w.gamma, opt)
        try:
            nll, grad, st = F.fsa_nll_grad(ctx, None, True)
        finally:
            F.fsa_destroy(ctx)
        return nll, grad, st

    for _ in range(warmup):
        step(options(0))
    prof = step(options(F.PROFILE_ALL))[2]
    dom = int(np.argmax(prof["kernel_ms"][:4]))
    opt = options(1 << dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [step(opt) for _ in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    probe_iters = sum(o[2]["probe_iters"] for o in outs)
    kms = np.sum([o[2]["kernel_ms"] for o in outs], axis=0)
    kcnt = np.sum([o[2]["kernel_launches"] for o in outs], axis=0)
    pcg_ms = sum(o[2]["ms_pcg"] for o in outs)
    return {
        "value": probe_iters / dt,
        "ms_per_step": 1000.0 * dt / steps,
        "pcg_only_probe_iters_per_s": probe_iters / (pcg_ms / 1000.0),
        "probe_iters_per_step": probe_iters / steps,
        "iters": [outs[-1][2]["iters_min"], outs[-1][2]["iters_max"]],
        "nll": outs[-1][0],
        "grad": [float(g) for g in outs[-1][1]],
        "ms_build": float(np.mean([o[2]["ms_build"] for o in outs])),
        "ms_pcg": pcg_ms / steps,
        "ms_backward": float(np.mean([o[2]["ms_backward"] for o in outs])),
        "nnz": outs[-1][2]["nnz"],
        "dominant_class": dom,
        "kernel_ms": kms.tolist(),
        "kernel_launches": kcnt.tolist(),
        "profiled_step_kernel_ms": list(prof["kernel_ms"]),
        "profiled_step_kernel_launches": list(prof["kernel_launches"]),
    }


def roofline(res, n, m, tp, precision):
    """precision: "f64", "f32" (float32 operator) or "bf16a" (float32
    operator whose low-rank passes read A in bfloat16 and run on the
    bfloat16 MFMA; their peak is the bfloat16 one, the other kernels'
    the float32 one)."""
    b = 8 if precision == "f64" else 4
    ba = 2 if precision == "bf16a" else b
    dom = res["dominant_class"]
    avg = [res["profiled_step_kernel_ms"][k] / max(res["profiled_step_kernel_launches"][k], 1) for k in range(5)]
    avg[dom] = res["kernel_ms"][dom] / max(res["kernel_launches"][dom], 1)  # over the timed steps

    def bound(k):
        """(bound, achieved, peak, unit, frac, bytes, flops, GB/s, TFLOP/s) of class k at its average launch"""
        byt, flop = kernel_work(k, n, m, tp, res["nnz"], b, ba)
        t_s = max(avg[k], 1e-9) / 1000.0
        gbs, tfl = byt / t_s / 1e9, flop / t_s / 1e12
        peak_t = PEAK_TFLOPS["f64" if precision == "f64" else ("bf16" if precision == "bf16a" and k in (1, 2) else "f32")]
        if flop / (peak_t * 1e12) > byt / (HBM_PEAK_GBS * 1e9):
            return "mfma", tfl, peak_t, "TFLOP/s", tfl / peak_t, byt, flop, gbs, tfl
        return "hbm", gbs, HBM_PEAK_GBS, "GB/s", gbs / HBM_PEAK_GBS, byt, flop, gbs, tfl

    bnd, ach, peak, unit, frac, byt, flop, gbs, tfl = bound(dom)
    r = {"bound": bnd, "achieved": ach, "peak": peak, "unit": unit, "frac": frac}
    name = KERNEL_NAMES[precision][dom]
    r.update({"traffic": measured_traffic(name), "kernel": KERNELS[dom], "rocprof_kernel": name,
              "avg_launch_ms": avg[dom], "algorithmic_bytes": byt, "algorithmic_flops": flop, "achieved_GBps": gbs,
              "achieved_TFLOPs": tfl, "source_fingerprint": source_fingerprint(),
              "per_kernel_avg_ms": dict(zip(KERNELS, avg)),
              "per_kernel_frac": {KERNELS[k]: {"bound": bound(k)[0], "frac": bound(k)[4]} for k in range(4)},
              "timing": "the dominant kernel class timed with HIP events over the timed steps; the other classes "
                        "from one untimed step with every class timed"})
    return r


def run_vecchia(F, torch, n, mv, m, t, steps, warmup, seed=0, cpu_sample_n=0):
    """The Vecchia path with the FITC preconditioner (Section 5) at the size
    of its experiments: n points uniform on the unit square, m_v nearest
    earlier neighbours, m kmeans++ inducing points, Matern-3/2 with rho =
    0.05, W uniform on [0.05, 0.25] (a Bernoulli-logit Hessian's range), t
    probes; a step is one solve + SLQ log det (one block PCG run)."""
    from workloads import generators as G
    locs = G.uniform_locations(n, seed + 100)
    ind = G.kmeanspp_inducing(locs, m, seed + 101)
    wts = G.laplace_weights(n, seed + 102)
    rhs = np.random.default_rng(seed + 103).standard_normal(n)
    d = {k: torch.from_numpy(np.ascontiguousarray(a)).cuda() for k, a in
         (("locs", locs), ("ind", ind), ("w", wts), ("rhs", rhs))}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v = F.Vecchia(d["locs"], d["ind"], F.MATERN32, 1.0, 0.05, mv, d["w"])
    torch.cuda.synchronize()
    ms_build = (time.perf_counter() - t0) * 1e3
    for i in range(warmup):
        v.solve_logdet(d["rhs"], t, i, tol=1e-6, max_iter=3000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, lds = 0, []
    for i in range(steps):
        _, ld, st = v.solve_logdet(d["rhs"], t, 1000 + i, tol=1e-6, max_iter=3000)
        its += st["probe_iters"]
        lds.append(ld)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    # the dominant kernels: the level-scheduled triangular solves of one
    # Sigma_V product on t+1 columns, timed with HIP events on the stream the
    # library runs on (torch's current stream, given at build)
    X = torch.randn(n, t + 1, dtype=torch.float64, device="cuda")
    v.apply(F.V_SIGMA, X)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        v.apply(F.V_SIGMA, X)
    e1.record()
    torch.cuda.synchronize()
    ms_prod = e0.elapsed_time(e1) / 3
    nnz_b = n * mv - mv * (mv + 1) // 2  # sum over i of min(m_v, i)
    # per pass: each list entry (4 B index, 8 B coefficient, a gathered row of
    # t+1 doubles) and each point's own row read and written
    prod_bytes = 2 * (nnz_b * (12 + 8 * (t + 1)) + n * 16 * (t + 1))
    v.close()
    out = {"workload": f"vecchia_solve_logdet n={n} m_v={mv} m={m} t={t} matern32 rho=0.05 W~U[0.05,0.25] tol=1e-6",
           "value": its / sec, "unit": "probe-iters/s", "ms_per_step": sec * 1e3 / steps, "ms_build": ms_build,
           "probe_iters_per_step": its / steps, "iters_max": st["iters_max"], "nlevels": st["nlevels"],
           "logdet": lds[-1], "logdet_spread": float(np.std(lds)) if len(lds) > 1 else 0.0, "steps": steps,
           "roofline": {"bound": "hbm", "achieved": prod_bytes / (ms_prod * 1e-3) / 1e9, "peak": 8000.0, "unit": "GB/s",
                        "frac": prod_bytes / (ms_prod * 1e-3) / 1e9 / 8000.0, "traffic": None,
                        "kernel": "Sigma_V product (k_vtri, both passes)", "ms_per_product": ms_prod,
                        "algorithmic_bytes": prod_bytes,
                        "note": f"latency-bound: {st['nlevels']} dependent levels per pass, one launch each"}}
    if cpu_sample_n:
        # The first ns points of the ordered workload are a Vecchia model of
        # their own (their neighbours are earlier points): the oracle solves
        # it and its rate is scaled by ns / n (per-iteration cost linear in n).
        from oracle import vecchia_oracle as VO
        ns = min(cpu_sample_n, n)
        tb = time.perf_counter()
        mdl = VO.Vecchia(locs[:ns], ind, (F.MATERN32, 1.0, 0.05), mv, wts[:ns])
        ts = time.perf_counter()
        o = VO.solve_logdet(mdl, rhs[:ns], t, seed=1000, tol=1e-6, max_iter=3000)
        te = time.perf_counter()
        rate = float(o["iters"].sum()) / (te - ts)
        try:
            from threadpoolctl import threadpool_info
            cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
        except Exception:
            cores = os.cpu_count() or 1
        out["cpu_baseline"] = {
            "value": rate * ns / n, "unit": "probe-iters/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"oracle solve + SLQ log det on the first {ns} points of the same ordered workload (a Vecchia "
                       f"model of its own), {int(o['iters'].sum())} probe-iterations; rate {rate:.1f} probe-iters/s "
                       f"at n={ns} scaled by {ns}/{n}; oracle build {ts - tb:.1f} s not included; its dense "
                       f"products run on {int(cores)} BLAS threads, its triangular solves (scipy) on one")}
    return out


def run_serving(F, torch, n_requests, rate, slots, budget_gib, warm=8, legs=("mixed", "fp64", "capacity"),
                graph=True):
    """The serving stream: `n_requests` likelihood + gradient (70%) and
    predictive-variance (30%) requests with Poisson arrivals at `rate` per
    second, n log-uniform in [5k, 300k], m in {100, 200, 500}, t = 20, through
    the library's server (mixed precision, `slots` workers, admission against
    `budget_gib` GiB), and the same trace through a one-at-a-time float64
    server (one worker).  solves/s = completed requests / (last completion -
    first arrival); latency = completion - arrival."""
    from workloads import configs
    from workloads import generators as G
    trace = configs.serving_trace(n_requests, rate)
    t0 = time.perf_counter()
    resp = G.rff_response_torch(torch)
    arrays = [r.materialize(256, response=resp) for r in trace]
    log(f"serving inputs ready in {time.perf_counter() - t0:.1f} s ({n_requests} requests)")

    def submit(srv, r, a, at):
        locs, y, ind, pred = a
        kind = F.REQ_NLL_GRAD if r.kind == "nll_grad" else F.REQ_PREDICT_VAR
        return srv.submit(kind, locs, y, r.theta, ind, r.gamma, pred, r.num_samples, arrival_ms=at)

    def one(label, precision, nslots, tol, graph, paced=True):
        opts = dict(num_probes=20, seed=4005, tol=tol, max_iter=2000, precision=precision, rr_period=20, graph=graph)
        with F.Server(slots=nslots, hbm_budget=int(budget_gib * (1 << 30)), **opts) as srv:
            for r, a in zip(trace[:warm], arrays[:warm]):  # code objects, library handles, pinned blocks
                srv.wait(submit(srv, r, a, 0.0))
            start = srv.clock_ms() + 100.0
            ids = [submit(srv, r, a, start + (1000.0 * r.arrival_s if paced else 0.0)) for r, a in zip(trace, arrays)]
            res = []
            for k, i in enumerate(ids):
                res.append(srv.wait(i)[0])
                if (k + 1) % 128 == 0:
                    log(f"serving {label}: {k + 1}/{len(ids)} done")
            st = srv.stats()
        bad = [x for x in res if x["status"] not in (0, 4)]
        lat = np.array([x["done_ms"] - x["arrival_ms"] for x in res])
        kinds = np.array([r.kind for r in trace])
        span = max(x["done_ms"] for x in res) - min(x["arrival_ms"] for x in res)
        out = {"slots": nslots, "precision": label, "tol": tol, "graph": bool(graph),
               "arrivals": "poisson" if paced else "all at once (capacity)",
               "completed": len(res) - len(bad), "failed": len(bad),
               "solves_per_s": (len(res) - len(bad)) / (span / 1000.0), "makespan_s": span / 1000.0,
               "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
               "p50_ms_nll_grad": float(np.percentile(lat[kinds == "nll_grad"], 50)),
               "p50_ms_predict_var": float(np.percentile(lat[kinds == "predict_var"], 50)),
               "peak_active": st["peak_active"], "peak_reserved_GiB": st["peak_reserved"] / 2 ** 30,
               "budget_GiB": st["hbm_budget"] / 2 ** 30,
               "probe_iters": int(sum(x["probe_iters"] for x in res)),
               "max_peak_over_footprint": max(x["peak_bytes"] / x["footprint"] for x in res)}
        if bad:
            out["first_error"] = bad[0]["message"]
            for x in bad[:8]:
                r = trace[ids.index(x["id"])]
                log(f"  failed: {r.kind} n={r.n} m={r.m} footprint {x['footprint']} peak {x['peak_bytes']}: "
                    f"{x['message']}")
        log(f"serving {label}: {out['solves_per_s']:.1f} solves/s, p50 {out['p50_ms']:.1f} ms, "
            f"p99 {out['p99_ms']:.1f} ms, peak active {out['peak_active']}, failed {len(bad)}")
        return out

    if tuple(legs) != ("mixed", "fp64", "capacity"):
        # a subset of the legs (a profile of one of them): the legs' records only
        out = {"workload": f"serving stream: {n_requests} requests, legs {','.join(legs)}, graph {int(graph)}"}
        if "mixed" in legs:
            out["mixed"] = one("mixed_fp32", F.MIXED_FP32, slots, 1e-6, graph)
        if "fp64" in legs:
            out["fp64_one_at_a_time"] = one("fp64_one_at_a_time", F.FP64, 1, 1e-6, False)
        if "capacity" in legs:
            out["mixed_capacity"] = one("mixed_fp32", F.MIXED_FP32, slots, 1e-6, graph, paced=False)
        return out
    mixed = one("mixed_fp32", F.MIXED_FP32, slots, 1e-6, graph)
    base = one("fp64_one_at_a_time", F.FP64, 1, 1e-6, False)
    cap = one("mixed_fp32", F.MIXED_FP32, slots, 1e-6, graph, paced=False)
    return {"workload": f"serving stream: {n_requests} requests, Poisson {rate:g}/s, n log-uniform [5000, 300000], "
                        f"m in {{100, 200, 500}}, exponential or matern32, t=20, 70% nll+grad / 30% predict_var "
                        f"(n_p=n/4, s=20), tol=1e-6, budget {budget_gib:g} GiB",
            "metric": "serving solves/s and p50/p99 latency (ms)",
            "mixed": mixed, "fp64_one_at_a_time": base, "mixed_capacity": cap,
            "solves_per_s_ratio": mixed["solves_per_s"] / base["solves_per_s"],
            "p99_ratio": base["p99_ms"] / mixed["p99_ms"]}


def cpu_baseline(w, sample_n, iters):
    """The oracle on a spatial window of the same workload (same density,
    taper range, covariance and all m inducing points), `iters` PCG
    iterations on t+1 columns; the rate is scaled by sample_n / n to the
    full size (per-iteration cost is linear in n at fixed m and n_gamma)."""
    from oracle import fsa_oracle as O
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        blas_threads = os.cpu_count() or 1
    a = math.sqrt(sample_n / w.n)
    sel = (w.locs[:, 0] < a) & (w.locs[:, 1] < a)
    locs = w.locs[sel]
    y = w.y[sel]
    ns = locs.shape[0]
    t0 = time.perf_counter()
    mdl = O.FSA(locs, w.inducing, w.theta, w.gamma)
    t1 = time.perf_counter()
    Z = O.probes(mdl, w.num_probes, w.seed)
    B = np.column_stack([y, Z])
    t2 = time.perf_counter()
    O.pcg_lanczos(mdl.matvec, mdl.precond_solve, B, 0.0, iters, fixed_iter=iters)
    t3 = time.perf_counter()
    rate = B.shape[1] * iters / (t3 - t2)
    return {"value": rate * ns / w.n, "unit": "probe-iters/s", "cores": int(blas_threads), "kind": "oracle",
            "sample": (f"oracle PCG, {iters} iterations x {B.shape[1]} columns on the {ns}-point window "
                       f"[0,{a:.4f}]^2 of the same workload (all {w.m} inducing points, same gamma); rate "
                       f"{rate:.2f} probe-iters/s at n={ns} scaled by {ns}/{w.n}; oracle build "
                       f"{t1 - t0:.1f} s not included; its dense products run on {blas_threads} BLAS threads, "
                       f"its sparse products (scipy) on one"),
            "host_cores_visible": len(os.sched_getaffinity(0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=500_000)
    ap.add_argument("--m", type=int, default=500)
    ap.add_argument("--probes", type=int, default=50)
    ap.add_argument("--modes", default="fp64,fp64_tol6,mixed,mixed_mfma,bf16a",
                    help="comma list of fp64 (tolerance 1e-8, the accuracy reference), fp64_tol6 (float64 at the "
                         "mixed modes' tolerance 1e-6), mixed (float32 operator, float32 products of A split into "
                         "bfloat16 parts), mixed_mfma (the same on the float32 matrix cores), bf16a (float32 "
                         "operator, bfloat16 A)")
    ap.add_argument("--rr-period", type=int, default=20,
                    help="mixed modes: float64 residual replacement every this many iterations (0 = never)")
    ap.add_argument("--cpu-sample-n", type=int, default=80_000)
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-vecchia", action="store_true", help="skip the Vecchia (Section 5) leg")
    ap.add_argument("--vecchia-only", action="store_true", help="run only the Vecchia (Section 5) leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-stream leg")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving-stream leg")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-legs", default="mixed,fp64,capacity",
                    help="serving legs to run: mixed (paced), fp64 (one-at-a-time float64 loop), capacity (all queued)")
    ap.add_argument("--serve-graph", type=int, default=1,
                    help="mixed legs replay PCG iterations from HIP graphs (0: plain launches)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this size (for hardware-counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the library runs on one GPU "
              f"and does not shard the path across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2405_14492_amd import fsa as F
    from workloads import configs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    F.lib()
    if args.vecchia_only:
        log("vecchia leg")
        print(json.dumps({"vecchia": run_vecchia(F, torch, 100_000, 30, 200, args.probes, args.steps, args.warmup)}),
              flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": run_serving(F, torch, args.serve_requests, args.serve_rate, args.serve_slots,
                                                 args.serve_budget_gib, legs=args.serve_legs.split(","),
                                                 graph=bool(args.serve_graph))}), flush=True)
        return
    log(f"generating inputs n={args.n} m={args.m} t={args.probes}")
    t0 = time.perf_counter()
    w = configs.large_matern(n=args.n, m=args.m, t=args.probes)
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s; gamma={w.gamma:.6g}")
    dev = {"locs": torch.from_numpy(w.locs).cuda(), "y": torch.from_numpy(w.y).cuda(),
           "ind": torch.from_numpy(w.inducing).cuda()}
    torch.cuda.synchronize()
    if args.copy_calibration_mib:
        src = torch.empty(args.copy_calibration_mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration_mib} MiB read + written")
    results = {}
    for mode in args.modes.split(","):
        prec = {"mixed": F.MIXED_FP32, "mixed_mfma": F.MIXED_FP32, "bf16a": F.MIXED_BF16A, "fp64": F.FP64,
                "fp64_tol6": F.FP64}[mode]
        tol = 1e-8 if mode == "fp64" else 1e-6
        fp32p = F.F32P_MFMA if mode == "mixed_mfma" else F.F32P_SPLIT
        log(f"mode {mode}: warmup {args.warmup}, steps {args.steps}")
        results[mode] = run_mode(F, dev, w, prec, args.steps, args.warmup, tol, torch, args.rr_period, fp32p)
        log(f"mode {mode}: {results[mode]['value']:.1f} probe-iters/s, {results[mode]['ms_per_step']:.2f} ms/step, "
            f"iters {results[mode]['iters']}, kernel ms/launch "
            f"{[round(a / max(b, 1), 4) for a, b in zip(results[mode]['profiled_step_kernel_ms'], results[mode]['profiled_step_kernel_launches'])]}")
    main_mode = "mixed" if "mixed" in results else list(results)[0]
    r = results[main_mode]
    dtype = "f64" if main_mode in ("fp64", "fp64_tol6") else "f32"
    rkey = {"mixed": "f32", "mixed_mfma": "f32mfma", "bf16a": "bf16a", "fp64": "f64", "fp64_tol6": "f64"}[main_mode]
    out = {
        "metric": "PCG probe-iters/s at n=500k,m=500,t=50 (mixed precision; fp64 beside it)",
        "value": r["value"],
        "unit": "probe-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"fsa_nll_grad n={args.n} m={args.m} t={args.probes} matern32 "
                               f"rho=0.05 sigma2=0.1 n_gamma=80 tol={'1e-8' if main_mode == 'fp64' else '1e-6'}",
                   "n": args.n, "m": args.m, "t": args.probes, "gamma": w.gamma, "nnz": r["nnz"],
                   "rr_period": args.rr_period},
        "roofline": roofline(r, args.n, args.m, args.probes + 1, rkey),
        "pcg_only_probe_iters_per_s": r["pcg_only_probe_iters_per_s"],
        "modes": results,
    }
    if "fp64_tol6" in results and "mixed" in results:
        # the same PCG tolerance (1e-6) in both precisions: probe-iterations/s and time per likelihood step
        out["mixed_over_fp64_same_tol"] = results["mixed"]["value"] / results["fp64_tol6"]["value"]
        out["mixed_over_fp64_same_tol_pcg_only"] = (results["mixed"]["pcg_only_probe_iters_per_s"]
                                                    / results["fp64_tol6"]["pcg_only_probe_iters_per_s"])
        out["mixed_step_speedup_same_tol"] = results["fp64_tol6"]["ms_per_step"] / results["mixed"]["ms_per_step"]
        out["mixed_vs_fp64_same_tol_rel_nll"] = (abs(results["mixed"]["nll"] - results["fp64_tol6"]["nll"])
                                                 / abs(results["fp64_tol6"]["nll"]))
    if "fp64" in results and "mixed" in results:
        out["mixed_over_fp64"] = results["mixed"]["value"] / results["fp64"]["value"]
        out["mixed_over_fp64_pcg_only"] = (results["mixed"]["pcg_only_probe_iters_per_s"]
                                           / results["fp64"]["pcg_only_probe_iters_per_s"])
        out["mixed_step_speedup"] = results["fp64"]["ms_per_step"] / results["mixed"]["ms_per_step"]
        out["mixed_vs_fp64_rel_nll"] = abs(results["mixed"]["nll"] - results["fp64"]["nll"]) / abs(results["fp64"]["nll"])
        out["mixed_vs_fp64_rel_grad"] = [abs(a - c) / max(abs(c), 1e-300)
                                         for a, c in zip(results["mixed"]["grad"], results["fp64"]["grad"])]
        out["roofline_fp64"] = roofline(results["fp64"], args.n, args.m, args.probes + 1, "f64")
    if "mixed_mfma" in results:
        out["roofline_mixed_mfma"] = roofline(results["mixed_mfma"], args.n, args.m, args.probes + 1, "f32mfma")
        if "mixed" in results:
            out["split_over_mfma"] = results["mixed"]["value"] / results["mixed_mfma"]["value"]
    if "fp64" in results and "bf16a" in results:
        f, g = results["fp64"], results["bf16a"]
        out["bf16a_over_fp64"] = g["value"] / f["value"]
        out["bf16a_vs_fp64_rel_nll"] = abs(g["nll"] - f["nll"]) / abs(f["nll"])
        out["bf16a_vs_fp64_rel_grad"] = [abs(a - c) / max(abs(c), 1e-300) for a, c in zip(g["grad"], f["grad"])]
        out["roofline_bf16a"] = roofline(g, args.n, args.m, args.probes + 1, "bf16a")
    if not args.no_vecchia:
        log("vecchia leg (Section 5): n=100000 m_v=30 m=200")
        out["vecchia"] = run_vecchia(F, torch, 100_000, 30, 200, args.probes, args.steps, args.warmup,
                                     cpu_sample_n=0 if args.no_cpu_baseline else 15_000)
        log(f"vecchia: {out['vecchia']['value']:.1f} probe-iters/s, {out['vecchia']['ms_per_step']:.2f} ms/step, "
            f"{out['vecchia']['nlevels']} levels")
    if not args.no_serving:
        log("serving leg")
        out["serving"] = run_serving(F, torch, args.serve_requests, args.serve_rate, args.serve_slots,
                                     args.serve_budget_gib, legs=args.serve_legs.split(","),
                                     graph=bool(args.serve_graph))
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_n, args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
