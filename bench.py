#!/usr/bin/env python3
"""Benchmark of the minimizer on one MI355X.

Default workload: the FP64 hysteresis sweep on the 80 nm cube (40^3 Kuhn
cells: 68,921 magnet nodes, 250,047 potential nodes), field +8 -> -8 -> +8 T
in 0.1 T steps along z tilted by 1 degree, each point warm-started from the
previous minimum.  A "step" is a batch of --points-per-step (16) consecutive
field points of the loop (each a full minimization: trial steps, potential
solves, field, step logic, stopping test, continuation); --steps K times the
first 16 K points (default 20: 320 of the 321 points, both branches and both
switching fields).

Prints one JSON line with node-iterations/s (magnet nodes x energy-gradient
evaluations, line-search trials included, per second of wall time), the
roofline of the step kernel (algorithmic bytes of the method's per-row model
per launch over its average launch time, HIP events on the library's
stream), and in `detail` the same for one FP64 minimization of the
1.03M-node polycrystal (the pure-HBM case) and the p50/p99 latencies of a
bounded run of the served request stream; and the CPU oracle timed on a
bounded sample of the sweep.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-poly] [--no-serve] [--workload ...]
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node-iterations/s + HBM roofline fraction; served-solve p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def cpu_baseline(n_evals: int = 5) -> dict:
    """Time the oracle (one thread) on a prefix of the first field point of the
    same sweep: `n_evals` energy-gradient evaluations of its minimizer."""
    code = f"""
import os, sys, time, json
sys.path.insert(0, {ROOT!r})
from paper_1309_5796_amd import meshgen
import oracle
c = meshgen.config2()
s = oracle.System(c['mesh'])
t = time.perf_counter()
r = oracle.minimize(s, c['m0'], c['fields'][0], oracle.Options(max_evals={n_evals}))
dt = time.perf_counter() - t
print(json.dumps(dict(evals=r.evals, seconds=dt, N=s.N)))
"""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cmd = [sys.executable, "-c", code]
    if os.path.exists("/usr/bin/taskset"):
        cmd = ["taskset", "-c", "0"] + cmd
    out = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    if out.returncode != 0:
        return {"error": out.stderr[-500:]}
    d = json.loads(out.stdout.strip().splitlines()[-1])
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": d["N"] * d["evals"] / d["seconds"], "unit": "node-iterations/s", "cores": 1,
            "kind": "oracle",
            "sample": f"first {d['evals']} energy-gradient evaluations of the +8 T point of the same sweep "
                      f"(FP64 NumPy/SciPy, potential by Jacobi-CG to 1e-13), {d['seconds']:.1f} s on one core "
                      f"of {os.cpu_count()} ({cpu})"}


def kernel_source_hash() -> str:
    """Hash of the step kernel's source and of the host code that lays out its
    operands (layouts, lanes per row, block splits, the multigrid hierarchy):
    a change to any of them changes the traffic the counters measured.
    Comments and blank lines are left out (they change no code)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("paper_1309_5796_amd/csrc/kernels.hip", "paper_1309_5796_amd/csrc/device.h",
              "paper_1309_5796_amd/csrc/api.cpp", "paper_1309_5796_amd/csrc/amg.cpp"):
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines())
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()


def measured_traffic(name: str):
    """HBM bytes per launch from the committed counter runs (calibrated
    FETCH_SIZE + WRITE_SIZE), or None when the kernel source has changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    return rec["traffic_bytes_per_launch"] if rec.get("kernel_source_sha256") == kernel_source_hash() else None


def bytes_per_evaluation_model(sz: dict, evals: int, pcg_iters: int, fp64: bool = True) -> float:
    """Algorithmic HBM bytes of `evals` energy-gradient evaluations with
    `pcg_iters` potential-solver iterations in all, by the per-row model of
    the method's kernels (every matrix and vector touched once, gathered
    neighbours cached; int32 indices; z, z_L the measured average row
    lengths of the magnet pattern and of the potential matrix):
      FP64: per magnet node 296 + 64 z (divergence 36 + 28 z, field
            188 + 36 z, Cayley update 72); per potential row 44 + 12 z_L for
            the solve's start and 108 + 12 z_L per CG iteration;
      FP32 form: 156 + 36 z; 24 + 8 z_L; 56 + 8 z_L.
    With z = z_L = 15 this is B = 1256 N + (224 + 288 k) N_t per FP64
    evaluation (k CG iterations).  Preconditioner work beyond one Jacobi CG
    iteration is not counted: the model prices the method, not this
    implementation's multigrid."""
    N, Nt = sz["N"], sz["Nt"]
    z = sz["nnz_magnet"] / max(N, 1)
    zl = sz["nnz_potential"] / Nt if Nt else 0.0
    if fp64:
        node, init, it = 296 + 64 * z, 44 + 12 * zl, 108 + 12 * zl
    else:
        node, init, it = 156 + 36 * z, 24 + 8 * zl, 56 + 8 * zl
    return evals * (node * N + init * Nt) + pcg_iters * it * Nt


def roofline_of(tm, kernel, sz=None, evals=0, pcg_iters=0, fp64=True, traffic=None):
    """Roofline of the step kernel over a timed region.  `achieved` = the
    model's algorithmic bytes (bytes_per_evaluation_model) per launch over
    the average launch duration (HIP events bracketing every batch of step
    launches on the library's stream); `phase_model` gives the same for the
    library's per-phase byte table, which also counts every multigrid
    sweep."""
    if tm["launches"] <= 0 or tm["ms"] <= 0:
        return None
    secs = tm["ms"] / 1e3
    avg_s = secs / tm["launches"]
    out = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
           "traffic": traffic, "kernel": kernel, "avg_launch_us": avg_s * 1e6, "launches_timed": tm["launches"]}
    if sz is not None:
        B = bytes_per_evaluation_model(sz, evals, pcg_iters, fp64)
        out.update(achieved=B / secs / 1e9, frac=B / secs / 1e9 / HBM_PEAK_GBS,
                   alg_bytes_per_launch=B / tm["launches"],
                   alg_bytes_per_evaluation=B / max(evals, 1),
                   avg_row_lengths={"magnet": sz["nnz_magnet"] / max(sz["N"], 1),
                                    "potential": sz["nnz_potential"] / max(sz["Nt"], 1)})
    out["phase_model"] = {"achieved": tm["bytes"] / secs / 1e9, "frac": tm["bytes"] / secs / 1e9 / HBM_PEAK_GBS,
                          "alg_bytes_per_launch": tm["bytes"] / tm["launches"]}
    if traffic and sz is not None:
        out["traffic_over_alg"] = traffic / out["alg_bytes_per_launch"]
    return out


def base_line(value, K, warmup, wall, dtype, config):
    return {"metric": METRIC, "value": value, "unit": "node-iterations/s", "n_gpus": 1, "steps": K,
            "warmup": warmup, "ms_per_step": wall / max(K, 1) * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def poly_run(ctx, cfg, prec, max_evals):
    """One minimization of the polycrystal in one precision, with the
    library's kernel timing on."""
    import torch
    from paper_1309_5796_amd import binding
    t0 = time.perf_counter()
    p = binding.Problem(ctx, cfg["mesh"], precision=prec)
    setup = time.perf_counter() - t0
    sz = p.sizes()
    p.set_m(cfg["m0"])
    p.set_field(cfg["b_ext"])
    ctx.timing(True)
    ctx.timing_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = p.minimize(max_evals=max_evals)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = ctx.timing_read(reset=True)
    ctx.timing(False)
    p.close()
    name = "fp64" if prec == binding.FP64 else "mixed"
    print(f"[bench] polycrystal {name}: setup {setup:.1f} s, status {r.status} evals {r.evals} pcg {r.pcg_iters} "
          f"{wall:.2f} s E={r.energy_J:.12e} torque {r.max_torque:.2e}", file=sys.stderr, flush=True)
    return dict(r=r, wall=wall, tm=tm, sz=sz, setup=setup)


def poly_summary(o, fp64):
    r = o["r"]
    kernel = "k_step<double,4>" if fp64 else "k_step<float,4>"
    traffic = measured_traffic("k_step_fp64_poly") if fp64 else None
    return {"evals": r.evals, "iterations": r.iterations, "pcg_iters": r.pcg_iters, "wall_s": o["wall"],
            "setup_s": o["setup"], "status": r.status, "max_torque": r.max_torque, "energy_J": r.energy_J,
            "node_iterations_per_s": o["sz"]["N"] * r.evals / o["wall"],
            "roofline": roofline_of(o["tm"], kernel, o["sz"], r.evals, r.pcg_iters, fp64, traffic)}


def run_poly(args):
    """Config 3: 1.03M-node 64-grain polycrystal, one minimization at -2 T from
    +z + noise in the mixed form and in FP64; energies compared."""
    from paper_1309_5796_amd import binding, meshgen
    t0 = time.perf_counter()
    cfg = meshgen.config3()
    print(f"[bench] mesh {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    ctx = binding.Context(0)
    if args.lanes or args.blocks:
        ctx.set_launch_config(lanes_per_row=args.lanes, max_blocks=args.blocks)
    forms = [("mixed", binding.MIXED), ("fp64", binding.FP64)]
    if args.poly_prec != "both":
        forms = [f for f in forms if f[0] == args.poly_prec]
    out = {name: poly_run(ctx, cfg, prec, args.max_evals) for name, prec in forms}
    ctx.close()
    wl = "polycrystal, 200x200x100 nm box, 126x126x63 Kuhn cells, 64 grains, -2 T at 1 deg, one minimization"
    lead = "mixed" if "mixed" in out else "fp64"
    o = out[lead]
    line = base_line(o["sz"]["N"] * o["r"].evals / o["wall"], 1, 0, o["wall"],
                     "f64" if lead == "fp64" else "f32+f64-reductions",
                     {"workload": f"{lead} {wl}", "magnet_nodes": o["sz"]["N"], "potential_nodes": o["sz"]["Nt"]})
    line["roofline"] = poly_summary(o, lead == "fp64")["roofline"]
    line["detail"] = {name: poly_summary(v, name == "fp64") for name, v in out.items()}
    if len(out) == 2:
        fp = out["fp64"]["r"]
        scale = sum(abs(getattr(fp, k)) for k in ("e_exch_J", "e_anis_J", "e_zeem_J", "e_demag_J"))
        line["detail"]["rel_energy_mixed_vs_fp64"] = abs(out["mixed"]["r"].energy_J - fp.energy_J) / scale
    print(json.dumps(line), flush=True)


def run_grains(args):
    """Config 4: 256 independent grain cubes in the mixed form, one batched
    run (shared launches, autotuned shape) against the same solves one by one."""
    import numpy as np
    import torch
    from paper_1309_5796_amd import binding, meshgen
    t0 = time.perf_counter()
    cfgs = meshgen.config4(args.grains)
    print(f"[bench] {len(cfgs)} meshes {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    ctx = binding.Context(0)
    probs = []
    for c in cfgs:
        p = binding.Problem(ctx, c["mesh"], precision=binding.MIXED)
        p.set_m(c["m0"])
        p.set_field(c["b_ext"])
        probs.append(p)
    big = max(probs, key=lambda q: q.Nt)
    lanes, blocks, us = big.autotune()
    for p in probs:
        p.set_launch(lanes, blocks)
    states = [p.get_state() for p in probs]
    print(f"[bench] setup done, tuned lanes={lanes} blocks={blocks} ({us:.1f} us/launch)", file=sys.stderr, flush=True)
    Nsum = sum(p.N for p in probs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = binding.minimize_batch(probs)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    evals = sum(r.evals for r in res)
    node_evals = sum(p.N * r.evals for p, r in zip(probs, res))
    print(f"[bench] batch {t_batch:.1f} s", file=sys.stderr, flush=True)
    for p, st in zip(probs, states):
        p.set_state(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    single = []
    for k, p in enumerate(probs):
        single.append(p.minimize())
        if (k + 1) % 64 == 0:
            print(f"[bench] one by one {k + 1}/{len(probs)}: {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                  flush=True)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    # the shared launch runs small problems on fewer blocks than a lone run,
    # so the two agree to rounding (bitwise at equal launch shapes: tests)
    rel = [abs(a.energy_J - b.energy_J) / max(abs(b.e_exch_J) + abs(b.e_anis_J) + abs(b.e_zeem_J) + abs(b.e_demag_J),
                                                1e-300) for a, b in zip(res, single)]
    line = base_line(node_evals / t_batch, 1, 0, t_batch, "f32+f64-reductions",
                     {"workload": f"{len(probs)} grain cubes (edges log-uniform 10-60 nm), mixed precision, "
                                  f"-1 T, one batched run", "magnet_nodes_total": Nsum})
    line["roofline"] = None
    line["detail"] = {"batched_s": t_batch, "one_by_one_s": t_seq, "speedup": t_seq / t_batch,
                      "evals": evals, "max_rel_energy_diff_vs_one_by_one": float(max(rel)),
                      "tuned_lanes": lanes, "tuned_blocks": blocks,
                      "statuses": sorted(set(r.status for r in res))}
    for p in probs:
        p.close()
    ctx.close()
    print(json.dumps(line), flush=True)


def serve_stream(n_requests, hbm_gb, slots, timeout_s, log_every=15.0, rate_hz=200.0, assembly="host"):
    """Submit the first n_requests of the seeded 200 req/s Poisson stream at
    their arrival times to a server with an HBM budget; latency from each
    request's arrival time (its place in the stream) and from the return of
    its submit call (which only copies the request)."""
    import numpy as np
    from paper_1309_5796_amd import binding, meshgen
    reqs = meshgen.config5_requests(rate_hz=rate_hz)[:n_requests]
    t0 = time.perf_counter()
    built = [meshgen.request_mesh(r) for r in reqs]
    print(f"[bench] {len(built)} request meshes {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    ctx = binding.Context(0)
    if assembly == "device":
        ctx.set_assembly(binding.ASSEMBLE_DEVICE)
    srv = binding.Server(ctx, hbm_budget=int(hbm_gb * (1 << 30)), max_slots=slots)
    t_start = time.perf_counter()
    t_last = t_start
    pending = {}
    lat, lat_sub, node_evals, statuses, nodes, failed = [], [], 0.0, [], 0, []
    k = 0
    while k < len(reqs) or pending:
        now = time.perf_counter() - t_start
        while k < len(reqs) and reqs[k].arrival_s <= now:
            b = built[k]
            t = srv.submit(b["mesh"], b["b_ext"], precision=reqs[k].precision)
            pending[t] = (t_start + reqs[k].arrival_s, time.perf_counter(), meshgen.n_magnetic(b["mesh"]))
            k += 1
        for t in list(pending):
            try:
                got = srv.poll(t)
            except binding.MMSDError as e:   # a failed request: counted, not timed
                pending.pop(t)
                failed.append(e.code)
                continue
            if got is not None:
                r, _ = got
                t_arr, t_sub, n = pending.pop(t)
                lat.append(time.perf_counter() - t_arr)
                lat_sub.append(time.perf_counter() - t_sub)
                node_evals += n * r.evals
                nodes += n
                statuses.append(r.status)
        time.sleep(0.001)
        if time.perf_counter() - t_last > log_every:
            t_last = time.perf_counter()
            print(f"[bench] serve t={t_last - t_start:.0f} s submitted {k}/{len(reqs)} completed {len(lat)}",
                  file=sys.stderr, flush=True)
        if time.perf_counter() - t_start > timeout_s:
            print("[bench] serve timeout", file=sys.stderr, flush=True)
            break
    wall = time.perf_counter() - t_start
    st = srv.stats()
    srv.close()
    ctx.close()
    lat, lat_sub = np.array(lat), np.array(lat_sub)

    def pct(a, q):
        return float(np.percentile(a, q)) if len(a) else None

    return {"requests": len(reqs), "completed": int(len(lat)), "wall_s": wall,
            "node_iterations_per_s": node_evals / wall, "magnet_nodes_completed": nodes,
            "p50_s": pct(lat, 50), "p99_s": pct(lat, 99),
            "p50_from_submit_s": pct(lat_sub, 50), "p99_from_submit_s": pct(lat_sub, 99),
            "statuses": sorted(set(statuses)), "failed": len(failed), "failed_codes": sorted(set(failed)),
            "device_launches": st["launches"],
            "setup_seconds_summed": st["setup_seconds"], "device_loop_busy_s": st["loop_seconds"],
            "offered_rate_req_s": rate_hz, "served_rate_req_s": len(lat) / wall, "assembly": assembly,
            "hbm_budget_GB": hbm_gb, "slots": slots}


def run_serve(args):
    """Config 5: the first --requests of the seeded Poisson stream (200 req/s)
    submitted at their arrival times to a server with an HBM budget; reports
    arrival-to-result latency percentiles (and from the submit call's
    return) and node-iterations/s."""
    d = serve_stream(args.requests, args.hbm_gb, args.slots, args.serve_timeout, rate_hz=args.rate,
                     assembly=args.assembly)
    line = base_line(d["node_iterations_per_s"], d["completed"], 0, d["wall_s"], "mixed f64/f32 per request",
                     {"workload": f"served minimizations: first {d['requests']} requests of the seeded {args.rate:g} req/s "
                                  f"Poisson stream, 2:2:1 boxes 1.2k-520k nodes, 64-grain density, "
                                  f"B ~ U(-4,4) T, FP64/mixed coin", "hbm_budget_GB": args.hbm_gb,
                      "slots": args.slots})
    line["roofline"] = None
    line["detail"] = d
    print(json.dumps(line), flush=True)


def run_sphere(args):
    """The paper's experiment analog (Results, comparison with the LLG
    solver): 20 nm Nd2Fe14B sphere (staircase Kuhn ball, 85k magnetic tets),
    FP64, field 0 -> -6 T in 0.01 T steps at 45 degrees, each point warm
    started; the coercive field is bisected to 1e-4 T and compared with half
    the anisotropy field (the Stoner-Wohlfarth value at 45 degrees); the
    evaluation count is the sweep's (the paper: 13,250 for its stopping test)."""
    import numpy as np
    import torch
    from paper_1309_5796_amd import binding, meshgen
    t0 = time.perf_counter()
    cfg = meshgen.sphere_experiment()
    ctx = binding.Context(0)
    p = binding.Problem(ctx, cfg["mesh"], precision=binding.FP64)
    p.set_m(cfg["m0"])
    print(f"[bench] sphere setup {time.perf_counter() - t0:.1f} s: {p.N} magnet / {p.Nt} potential nodes",
          file=sys.stderr, flush=True)
    fields = cfg["fields"]
    stop = binding.STOP_SUM_SQ if args.stop == "sumsq" else binding.STOP_MAX_TORQUE
    res, bsw = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k0 in range(0, len(fields), args.chunk * 5):
        r_chunk, b_chunk = p.hysteresis(fields[k0:k0 + args.chunk * 5], refine_tol_T=1e-4, stop_rule=stop)
        res.extend(r_chunk)
        bsw.extend(float(b) for b in b_chunk)
        print(f"[bench] sphere field points {len(res)}/{len(fields)}: {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    evals = sum(r.evals for r in res)
    hk_half = meshgen.K1_JM3 * 4e-7 * np.pi / meshgen.JS_T      # mu0 H_K / 2 = K1 / Ms
    # a switching inside a chunk is bisected there; one at a chunk boundary
    # is seen from the projections
    proj = np.array([float(np.dot(r.m_avg, -meshgen.U_H_45DEG)) for r in res])
    flips = [k for k in range(1, len(proj)) if np.sign(proj[k]) != np.sign(proj[k - 1])]
    hc = bsw[0] if bsw else ((flips[0] - 0.5) * 0.01 if flips else None)
    line = base_line(p.N * evals / wall, len(fields), 0, wall, "f64",
                     {"workload": "20 nm sphere (85k-tet Kuhn ball), FP64, 0 -> -6 T in 0.01 T at 45 deg",
                      "magnet_nodes": p.N, "potential_nodes": p.Nt,
                      "stopping_test": "sum of squared torques < 1e-12 (the paper's)" if args.stop == "sumsq"
                      else "max torque < 1e-6"})
    line["roofline"] = None
    line["detail"] = {"evals": evals, "iterations": sum(r.iterations for r in res),
                      "pcg_iters": sum(r.pcg_iters for r in res), "wall_s": wall,
                      "coercive_field_T": hc, "half_anisotropy_field_T": hk_half,
                      "rel_error": abs(hc - hk_half) / hk_half if hc else None,
                      "paper_evaluations": 13250, "paper_rel_error": 6e-4,
                      "statuses": sorted(set(r.status for r in res))}
    p.close()
    ctx.close()
    print(json.dumps(line), flush=True)


def run_ablation(args):
    """Step-length rules (eq. (10) and the adaptive switch the paper adopts):
    energy-gradient evaluations per rule on config 1 (one minimization) and
    on the whole FP64 loop of the 80 nm cube (321 points)."""
    import numpy as np
    import torch
    from paper_1309_5796_amd import binding, meshgen
    rules = [("adaptive", binding.STEP_ADAPTIVE), ("alternate", binding.STEP_ALTERNATE),
             ("bb1", binding.STEP_BB1), ("bb2", binding.STEP_BB2)]
    ctx = binding.Context(0)
    c1 = meshgen.config1()
    c2 = meshgen.config2()
    out = {}
    p1 = binding.Problem(ctx, c1["mesh"])
    p2 = binding.Problem(ctx, c2["mesh"])
    s2 = p2.get_state()
    npts = min(args.ablation_points, len(c2["fields"]))
    for name, rule in rules:
        p1.set_m(c1["m0"])
        p1.set_field(c1["b_ext"])
        r1 = p1.minimize(step_rule=rule)
        p2.set_state(s2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, bsw = p2.hysteresis(c2["fields"][:npts], step_rule=rule)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        proj = [float(np.dot(r.m_avg, meshgen.U_H_1DEG)) for r in res]
        bu = c2["fields"][:npts] @ meshgen.U_H_1DEG
        sw = [0.5 * (bu[k - 1] + bu[k]) for k in range(1, npts) if np.sign(proj[k]) != np.sign(proj[k - 1])]
        out[name] = {"config1_evals": r1.evals, "config1_iterations": r1.iterations, "config1_status": r1.status,
                     "sweep_evals": sum(r.evals for r in res), "sweep_iterations": sum(r.iterations for r in res),
                     "sweep_pcg_iters": sum(r.pcg_iters for r in res), "sweep_wall_s": wall,
                     "sweep_statuses": sorted(set(r.status for r in res)), "switching_fields_T": sw}
        print(f"[bench] rule {name}: config1 {r1.evals} evals; sweep {out[name]['sweep_evals']} evals "
              f"{wall:.1f} s", file=sys.stderr, flush=True)
    p1.close()
    p2.close()
    ctx.close()
    print(json.dumps({"workload": f"step-rule ablation: config 1 minimization and the first {npts} points of "
                                  f"the 80 nm cube's FP64 loop", "detail": out}), flush=True)


def run_assemble(args):
    """Operator assembly of one mesh, host (mmsd_assembly_export) against
    device (mmsd_assemble_device: adjacency, patterns and values in kernels), wall time of
    one call each after an untimed size query and warm-up; on the largest
    request of the served stream (520k magnet / 1.25M potential nodes) and
    the 80 nm cube."""
    import ctypes as C
    import numpy as np
    import torch
    from paper_1309_5796_amd import binding, meshgen
    reqs = meshgen.config5_requests()[:60]
    meshes = [("served request (largest of the first 60)", meshgen.request_mesh(reqs[args.assemble_request])["mesh"]),
              ("80 nm cube", meshgen.config2()["mesh"])]
    ctx = binding.Context(0)
    lib = ctx.lib
    out = []
    for name, mesh in meshes:
        a = binding.MeshArgs(mesh)
        sizes = (C.c_int64 * 4)()
        binding._check(lib.mmsd_assembly_export(C.byref(a.c), a.mats, a.n_mats, sizes, *([None] * 12)))
        N, nnzM, Nt, nnzL = (int(x) for x in sizes)
        host = [np.empty(n) for n in (N + 1, nnzM, nnzM, 3 * nnzM, 3 * nnzM, 6 * N, N, Nt, Nt + 1, nnzL, nnzL, 4)]
        hp = [x.ctypes.data_as(C.c_void_p) for x in host]
        times_h, times_d = [], []
        for rep in range(3):
            t0 = time.perf_counter()
            binding._check(lib.mmsd_assembly_export(C.byref(a.c), a.mats, a.n_mats, sizes, *hp))
            times_h.append(time.perf_counter() - t0)
        dev = torch.device("cuda", 0)
        outs = [torch.empty(max(n, 1), dtype=torch.float64, device=dev)
                for n in (N + 1, nnzM, nnzM, 3 * nnzM, 3 * nnzM, 6 * N, N, Nt, Nt + 1, nnzL, nnzL)]
        dp = [C.c_void_p(t.data_ptr()) for t in outs]
        for rep in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            binding._check(lib.mmsd_assemble_device(ctx.handle, C.byref(a.c), a.mats, a.n_mats, sizes, *dp))
            torch.cuda.synchronize()
            times_d.append(time.perf_counter() - t0)
        print(f"[bench] assemble {name}: host {min(times_h):.3f} s, device {min(times_d):.3f} s",
              file=sys.stderr, flush=True)
        row = {"mesh": name, "magnet_nodes": N, "potential_nodes": Nt, "tets": int(mesh.tets.shape[0]),
               "host_s": min(times_h), "device_s": min(times_d)}
        del outs, host
        # whole problem creation (assembly, multigrid setup, device build),
        # FP64, with the operators from each assembly; best of two
        for where, flag in (("host", binding.ASSEMBLE_HOST), ("device", binding.ASSEMBLE_DEVICE)):
            ctx.set_assembly(flag)
            best = None
            for rep in range(2):
                t0 = time.perf_counter()
                p = binding.Problem(ctx, mesh)
                wall = time.perf_counter() - t0
                t = p.setup_times()
                t["wall"] = wall
                p.close()
                if best is None or t["total"] < best["total"]:
                    best = t
            row[f"create_{where}_assembly"] = best
            print(f"[bench] create {name} with {where} assembly: " +
                  ", ".join(f"{k} {v:.3f}" for k, v in best.items()), file=sys.stderr, flush=True)
        ctx.set_assembly(binding.ASSEMBLE_HOST)
        out.append(row)
    ctx.close()
    print(json.dumps({"workload": "operator assembly, host vs device", "host_threads":
                      min(16, os.cpu_count() or 1), "detail": out}), flush=True)


def run_copy(args):
    """Counter calibration: a plain 256 MiB device copy (read 256 MiB, write 256 MiB)."""
    from paper_1309_5796_amd import binding
    ctx = binding.Context(0)
    nbytes = 256 << 20
    ms = ctx.copy_probe(nbytes, reps=10)
    print(json.dumps({"workload": "copy probe", "bytes_read": nbytes, "bytes_written": nbytes,
                      "ms": ms, "GBps": 2 * nbytes / ms / 1e6}), flush=True)
    ctx.close()


def run_sweep(args):
    """The FP64 hysteresis loop of the 80 nm cube, K steps of `points_per_step`
    field points each, timed; returns the line's pieces."""
    import numpy as np
    import torch
    from paper_1309_5796_amd import binding, meshgen

    cfg = meshgen.config2()
    fields = cfg["fields"]
    P = max(1, args.points_per_step)
    K = max(1, args.steps)
    npts = min(K * P, len(fields))
    ctx = binding.Context(0)
    if args.lanes or args.blocks:
        ctx.set_launch_config(lanes_per_row=args.lanes, max_blocks=args.blocks)
    if args.vcycle == "plain":
        ctx.set_vcycle(0)
    p = binding.Problem(ctx, cfg["mesh"], precision=binding.FP64)
    sz = p.sizes()
    state0 = p.get_state()
    pc = {"auto": binding.PRECOND_AUTO, "jacobi": binding.PRECOND_JACOBI, "amg": binding.PRECOND_AMG}[args.precond]
    if args.warmup > 0:
        for w in range(args.warmup):
            p.hysteresis(fields[(w * P) % len(fields):(w * P) % len(fields) + P], precond=pc)
        p.set_state(state0)
    ctx.timing(not args.no_kernel_timing)
    ctx.timing_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for k in range(K):
        lo = k * P
        if lo >= len(fields):
            break
        r_chunk, _ = p.hysteresis(fields[lo:min(npts, lo + P)], precond=pc)
        res.extend(r_chunk)
        if (k + 1) % 4 == 0 or k + 1 == K:
            print(f"[bench] step {k + 1}/{K}: field points {len(res)}/{npts}, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # switching: first sign change of <m>.u_H along each branch (bracket midpoint)
    proj = [float(np.dot(r.m_avg, meshgen.U_H_1DEG)) for r in res]
    bu = fields[:npts] @ meshgen.U_H_1DEG
    bsw = [0.5 * (bu[k - 1] + bu[k]) for k in range(1, npts) if np.sign(proj[k]) != np.sign(proj[k - 1])]
    tm = ctx.timing_read(reset=True)
    ctx.timing(False)
    p.close()
    ctx.close()
    wall = t1 - t0
    evals = sum(r.evals for r in res)
    pcg = sum(r.pcg_iters for r in res)
    roof = None
    if not args.no_kernel_timing:
        roof = roofline_of(tm, f"k_step<double,{args.lanes or 4}>", sz, evals, pcg, True,
                           measured_traffic("k_step_fp64_sweep80"))
        if roof:
            roof["memory_level"] = ("hbm-or-mall: the cube's working set (~290 MB with the multigrid hierarchy) "
                                    "is largely resident in the 256 MB Infinity Cache")
    b0, b1 = float(bu[0]), float(bu[npts - 1])
    desc = "whole loop" if npts == len(fields) else f"first {npts} of the {len(fields)}-point loop"
    config = {"workload": f"FP64 hysteresis sweep, 80 nm cube, 40^3 Kuhn cells ({sz['N']:,} magnet / "
                          f"{sz['Nt']:,} potential nodes): field {b0:+.1f} T -> ... -> {b1:+.1f} T in 0.1 T steps "
                          f"at 1 deg ({desc} +8 -> -8 -> +8 T), {P} field points per step",
              "field_points": npts, "points_per_step": P, "magnet_nodes": sz["N"], "potential_nodes": sz["Nt"],
              "potential_preconditioner": args.precond, "vcycle": args.vcycle}
    detail = {"evals": evals, "iterations": sum(r.iterations for r in res), "pcg_iters": pcg,
              "pcg_iters_per_eval": pcg / max(evals, 1), "launches": sum(r.launches for r in res),
              "wall_s": wall, "switching_fields_T": [float(x) for x in bsw],
              "statuses": sorted(set(r.status for r in res))}
    return sz["N"] * evals / wall, K, wall, config, roof, detail


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="steps timed; a step is --points-per-step field points of the loop (20 x 16 = 320 of "
                         "the 321 points: both branches and both switching fields)")
    ap.add_argument("--points-per-step", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-poly", action="store_true", help="leave the polycrystal FP64 run out of the default line")
    ap.add_argument("--no-serve", action="store_true", help="leave the bounded serve out of the default line")
    ap.add_argument("--serve-requests", type=int, default=24,
                    help="requests of the stream the default line's bounded serve runs")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--blocks", type=int, default=0, help="blocks per problem (multiple of 8; 0 = library default)")
    ap.add_argument("--chunk", type=int, default=20, help="field points per library call (sphere)")
    ap.add_argument("--workload", default="sweep80",
                    choices=["sweep80", "poly", "grains", "serve", "sphere", "copy", "assemble", "ablation"])
    ap.add_argument("--stop", default="max", choices=["max", "sumsq"],
                    help="stopping test of --workload sphere: max torque < 1e-6 or the paper's sum of squares")
    ap.add_argument("--ablation-points", type=int, default=321)
    ap.add_argument("--assemble-request", type=int, default=38,
                    help="request of the served stream whose mesh --workload assemble times")
    ap.add_argument("--max-evals", type=int, default=100000)
    ap.add_argument("--grains", type=int, default=256)
    ap.add_argument("--requests", type=int, default=60)
    ap.add_argument("--hbm-gb", type=float, default=64.0)
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--serve-timeout", type=float, default=900.0)
    ap.add_argument("--rate", type=float, default=200.0, help="arrival rate of the served stream (req/s)")
    ap.add_argument("--assembly", default="host", choices=["host", "device"],
                    help="where served requests assemble their operators")
    ap.add_argument("--poly-prec", default="both", choices=["both", "mixed", "fp64"])
    ap.add_argument("--precond", default="auto", choices=["auto", "jacobi", "amg"],
                    help="preconditioner of the potential solve")
    ap.add_argument("--vcycle", default="fused", choices=["fused", "plain"],
                    help="multigrid cycle: restriction and coarse solve fused into the down-sweep "
                         "where the library finds it pays (default), or the plain order")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is "
              f"described but not built", file=sys.stderr)
        sys.exit(2)
    if args.workload != "sweep80":
        {"poly": run_poly, "grains": run_grains, "serve": run_serve, "sphere": run_sphere,
         "copy": run_copy, "assemble": run_assemble, "ablation": run_ablation}[args.workload](args)
        return

    value, K, wall, config, roof, detail = run_sweep(args)
    line = base_line(value, K, args.warmup, wall, "f64", config)
    line["roofline"] = roof
    line["detail"] = detail
    if not args.no_poly:
        # the headline HBM case: 1.03M magnet / 2.17M potential nodes, far
        # above the Infinity Cache; one FP64 minimization, untimed by the line
        from paper_1309_5796_amd import binding, meshgen
        t0 = time.perf_counter()
        cfg3 = meshgen.config3()
        print(f"[bench] polycrystal mesh {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        ctx = binding.Context(0)
        o = poly_run(ctx, cfg3, binding.FP64, args.max_evals)
        ctx.close()
        del cfg3
        d = poly_summary(o, True)
        d["workload"] = ("FP64 polycrystal, 200x200x100 nm, 126x126x63 Kuhn cells, 64 grains "
                         f"({o['sz']['N']:,} magnet / {o['sz']['Nt']:,} potential nodes), -2 T, one minimization")
        line["detail"]["polycrystal_fp64"] = d
    if not args.no_serve:
        d = serve_stream(args.serve_requests, args.hbm_gb, args.slots, args.serve_timeout)
        d["workload"] = (f"served minimizations: first {d['requests']} requests of the seeded 200 req/s Poisson "
                         f"stream (2:2:1 boxes, FP64/mixed coin)")
        line["detail"]["serve"] = d
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
