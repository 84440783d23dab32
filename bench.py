"""Throughput of the LB-SMRT collide-and-stream step on one MI355X.

Workload (default): 256^3 periodic box, D3Q343 (tensor product of the D1Q7
rule r*{0,+-1,+-2,+-3}, degree 9), Hermite order N = 4, Kn = 0.05, Maxwellian
perturbed by 16 random Fourier modes per field, FP32 state and contractions,
FP64 conserved moments / frame shift / relaxation.

Prints one JSON line: MLUPS (interior node updates per second / 1e6), the
roofline of the step kernel (HBM bound: one FP32 read and one FP32 write of
every population per node-step = 8 Q bytes; beside the nominal peak, a plain
device copy of one state buffer measured in the same run), the FP64 CPU oracle
timed on a bounded sample of the same workload, and variants of the same box:
the other contraction forms (FP32 on the vector units, split-BF16x3 on the matrix
cores, with its bf16 matrix-core flop rate), the additive collision, the moment-state form
of the step (state held as the M moments), the adjoint step, the Ma 3 D3Q729
calibration shock and the batched 64-shock Mach sweep.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0   # dense bf16 matrix-core peak of the MI355X
PRECISIONS = ("fp64_contract", "fp32", "split_bf16x3")

WORKLOADS = {
    # name: (abscissae, degree, N, box edge)
    "box256_q343_n4": ([1, 2, 3], 9, 4, 256),
    "box128_q343_n4": ([1, 2, 3], 9, 4, 128),
    "box160_q729_n5": ([1, 2, 3, 5], 11, 5, 160),
}

TAU_STAR = {(2, 0): 1.0, (2, 1): 1.0, (3, 0): 2 / 3, (3, 1): 3 / 2, (4, 0): 432 / 763, (4, 1): 6 / 7,
            (4, 2): 3 / 2, (5, 0): 864 / 1655, (5, 1): 108 / 163, (5, 2): 1.0}   # Table 4


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_k_collide_stream_box256_q343_n4.md")


def kernel_source_digest():
    """sha256 over the HIP sources and the C header, in a fixed order: the key under which
    the HBM traffic counters of the step kernel were recorded."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2401_11086_amd", "csrc")
    files = sorted(os.path.join(csrc, n) for n in os.listdir(csrc) if n.endswith((".hpp", ".hip", ".cpp")))
    for path in files + [os.path.join(ROOT, "include", "lbsmrt.h")]:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(workload, precision):
    """HBM bytes per launch of the step kernel from the committed FETCH_SIZE / WRITE_SIZE counter
    summary, if it was taken on this workload and precision with the current sources; else None.
    The summary's `- key: value` lines hold `workload`, `source_sha256` and, per precision P,
    `traffic_bytes_per_launch[P]`."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            kv = dict(ln[2:].split(": ", 1) for ln in fh.read().splitlines() if ln.startswith("- ") and ": " in ln)
        if kv.get("workload") != workload or kv.get("source_sha256") != kernel_source_digest():
            return None
        return float(kv[f"traffic_bytes_per_launch[{precision}]"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(torch, ab, deg, N, edge, kn, sample_edge=32, steps=30):
    """The FP64 oracle on a sample_edge^3 box of the same Fourier workload (same modes and
    relaxation times), `steps` steps from the library's FP32 equilibrium state; MLUPS scaled
    from that sample.  The same steps on the GPU in each contraction precision, and in the
    moment-state form, give each form's error against the oracle (max |f_gpu - f_oracle| /
    max |f_oracle|, and the largest deviation of rho and theta)."""
    import numpy as np

    import oracle as O
    from paper_2401_11086_amd import Lattice
    from paper_2401_11086_amd import workloads as W
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(p.get("num_threads", 1)) for p in threadpool_info()] or [1])
    except Exception:
        threads = 1
    vs = O.make_velocity_set(ab, deg)
    tau20 = kn * edge * vs.r
    tau = {k: v * tau20 for k, v in TAU_STAR.items() if k[0] <= N}
    model = O.Model(vs=vs, N=N, tau=tau, shift=(0, 0, 0))
    dom = O.Domain(nx=sample_edge, ny=sample_edge, nz=sample_edge, bc_x=0)
    box = [dict(nx=sample_edge, ny=sample_edge, nz=sample_edge, bc_x=0)]
    n = sample_edge ** 3
    fields = torch.tensor(W.fourier_box(sample_edge), dtype=torch.float64, device="cuda")
    gpu = {}
    f32 = None
    for precision in PRECISIONS:
        lat = Lattice(ab, deg, N, tau, box, precision=precision)
        fa = lat.equilibrium(fields)
        if f32 is None:
            f32 = fa[:, :n].cpu().numpy()
        fb = lat.new_state()
        cur = lat.step(fa, fb, steps)
        lat.sync()
        gpu[precision] = cur[:, :n].double().cpu().numpy()
        if precision == "fp64_contract":
            # the moment-state form from the same state (its moments are the projection of it)
            ma = lat.project_state(lat.equilibrium(fields))
            mb, work = lat.new_moment_state(), lat.new_moment_work()
            m = lat.step_moment_state(ma, mb, work, steps)
            lat.sync()
            gpu["moment_state"] = lat.expand_state(m)[:, :n].double().cpu().numpy()
            del ma, mb, work, m
        lat.close()
    f = f32.astype(np.float64).reshape(vs.Q, sample_edge, sample_edge, sample_edge)
    t0 = time.perf_counter()
    for _ in range(steps):
        f = O.step(f, model, dom)
    dt = time.perf_counter() - t0
    assert np.isfinite(f).all()
    ref = f.reshape(vs.Q, n)
    ob_ref = O.observables(f, model, dom)
    errors = {}
    for precision, g in gpu.items():
        ob = O.observables(g.reshape(f.shape), model, dom)
        errors[precision] = {
            "f_max_scaled": float(np.abs(g - ref).max() / np.abs(ref).max()),
            "rho_max_abs": float(np.abs(ob["rho"] - ob_ref["rho"]).max()),
            "theta_max_abs": float(np.abs(ob["theta"] - ob_ref["theta"]).max())}
    # the same oracle on one thread, a few steps from the same state
    single = None
    try:
        from threadpoolctl import threadpool_limits
        f1 = f32.astype(np.float64).reshape(vs.Q, sample_edge, sample_edge, sample_edge)
        one_steps = 3
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            for _ in range(one_steps):
                f1 = O.step(f1, model, dom)
            dt1 = time.perf_counter() - t1
        single = {"value": round(n * one_steps / dt1 / 1e6, 6), "unit": "MLUPS", "cores": 1,
                  "sample": f"{sample_edge}^3 box, {one_steps} steps, {dt1:.1f} s"}
    except ImportError:
        pass
    return {"value": round(n * steps / dt / 1e6, 6), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{sample_edge}^3 periodic box of the same Fourier workload, {steps} steps, "
                      f"{dt:.1f} s; numpy FP64 with {threads} BLAS threads",
            "cpu_model": cpu_model(), "single_thread": single,
            "gpu_error_vs_oracle": errors}


def cpu_model():
    """The host CPU as /proc/cpuinfo names it (first processor: model name, family, model,
    stepping), with the logical CPUs this process may run on, or None."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if not line.strip():
                    break
                key, _, val = line.partition(":")
                fields[key.strip()] = val.strip()
    except OSError:
        return None
    if "model name" not in fields:
        return None
    ident = ", ".join(f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping") if k in fields)
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = None
    where = f"; {avail} of {os.cpu_count()} logical CPUs available to this process" if avail else ""
    return f"{fields['model name']} ({ident}{where})"


def shock_samples(torch):
    """The oracle and the GPU on two shock-tube workloads of the paper's set-up (Sec. 4.2),
    oracle steps bounded to a few seconds each: Ma 1.2, Nx 200, D3Q343, N = 4 (whole 1000-step
    run on the GPU, 100 oracle steps) and the Ma 3, Nx 600, D3Q729, N = 5 calibration tube
    (20 oracle steps).  MLUPS of each, on the same initial state."""
    import numpy as np

    import oracle as O
    from paper_2401_11086_amd import Lattice, solve_quadrature
    from paper_2401_11086_amd.shocks import shock_domain
    out = []
    for Ma, nx, ab, deg, N, gpu_steps, cpu_steps in ((1.2, 200, [1, 2, 3], 9, 4, 1000, 100),
                                                     (3.0, 600, [1, 2, 3, 5], 11, 5, 3000, 20)):
        c_l, _ = solve_quadrature(ab, deg)
        d, fields, st = shock_domain(Ma, nx, c_l)
        k = int(st["k"])
        tau = {key: v for key, v in TAU_STAR.items() if key[0] <= N}
        lat = Lattice(ab, deg, N, tau, [d], shift_k=(k, 0, 0), precision="fp64_contract")
        fa = lat.equilibrium(torch.tensor(fields, dtype=torch.float64, device="cuda"))
        f0 = fa[:, :nx].double().cpu().numpy()
        fb = lat.new_state()
        lat.step(fa, fb, 10)
        ms = _time_steps(torch, lambda: lat.step(fa, fb, gpu_steps), 1) / gpu_steps
        lat.sync()
        lanes = lat.launch_settings()["lanes_per_node"]
        lat.close()
        vs = O.make_velocity_set(ab, deg)
        model = O.Model(vs=vs, N=N, tau={key: v * d["tau_scale"] for key, v in tau.items()}, shift=(k, 0, 0))
        dom = O.Domain(nx=nx, bc_x=1, state_in=(d["rho_in"], d["u_in"], d["theta_in"]),
                       state_out=(d["rho_out"], d["u_out"], d["theta_out"]))
        f = f0.reshape(-1, 1, 1, nx)
        t0 = time.perf_counter()
        for _ in range(cpu_steps):
            f = O.step(f, model, dom)
        dt = time.perf_counter() - t0
        assert np.isfinite(f).all()
        out.append({"workload": f"Ma {Ma} shock, Nx {nx}, D3Q{vs.Q}, N={N}",
                    "oracle_mlups": round(nx * cpu_steps / dt / 1e6, 6), "oracle_steps": cpu_steps,
                    "gpu_mlups": round(nx / (ms / 1e3) / 1e6, 2), "gpu_steps": gpu_steps,
                    "gpu_lanes_per_node": lanes})
    return out


def device_record(torch):
    """Name, compute units and, where the driver exposes them, the current shader and memory
    clock levels of GPU 0 (read from sysfs; no helper program is started)."""
    import glob
    props = torch.cuda.get_device_properties(0)
    rec = {"name": props.name, "arch": getattr(props, "gcnArchName", None),
           "compute_units": props.multi_processor_count, "clocks": None}
    for dev in sorted(glob.glob("/sys/class/drm/card*/device")):
        try:
            clocks = {}
            for kind in ("sclk", "mclk"):
                with open(os.path.join(dev, f"pp_dpm_{kind}")) as fh:
                    cur = [ln.split(":", 1)[1].replace("*", "").strip() for ln in fh if ln.rstrip().endswith("*")]
                clocks[kind] = cur[0] if cur else None
            rec["clocks"] = clocks
            break
        except (OSError, IndexError):
            continue
    return rec


def copy_ceiling(torch, fa, fb, reps=5):
    """The HIP runtime's device copy of one state buffer into the other (same buffers, same run):
    the read + write rate a plain stream reaches on this GPU, beside the step kernel's."""
    fb.copy_(fa)
    torch.cuda.synchronize()
    ms = _time_steps(torch, lambda: fb.copy_(fa), reps)
    return 2.0 * fa.numel() * 4 / (ms / 1e3) / 1e9


def copy_calibration(torch, n_floats, steps, warmup):
    """Plain device-to-device copy of an f-sized float32 buffer: the achievable
    HBM rate for a read + write stream, and the reference for the traffic counters."""
    a = torch.ones(n_floats, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(max(warmup, 1)):
        b.copy_(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    gbs = 2.0 * 4 * n_floats / (ms / 1e3) / 1e9
    print(json.dumps({"metric": "device copy GB/s (read + write)", "value": round(gbs, 1), "unit": "GB/s",
                      "bytes_per_launch": 8 * n_floats, "ms_per_copy": round(ms, 4), "steps": steps}), flush=True)


def adjoint_pair(lat, f, lam_a, lam_b, dtau):
    """Two adjoint steps, each taking the other's output (timed as a dependent chain, as a reverse
    sweep runs them)."""
    lat.step_adjoint(f, lam_a, lam_b, dtau)
    lat.step_adjoint(f, lam_b, lam_a, dtau)


def _time_steps(torch, fn, n):
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(torch.cuda.current_stream())
    for _ in range(n):
        fn()
    ev1.record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / n


def time_variants(torch, lat, fa, fb, ab, deg, N, tau, edge, args, ms_fwd):
    """Same workload: the other contraction precision, and the adjoint step
    (lbsmrt_step_adjoint on its own, and with the forward replay a checkpointed
    reverse sweep adds per step)."""
    from paper_2401_11086_amd import Lattice
    out = {}
    steps = max(4, args.steps // 2)
    for other in [p for p in PRECISIONS if p != args.precision]:
        lat2 = Lattice(ab, deg, N, tau, [dict(nx=edge, ny=edge, nz=edge, bc_x=0)], precision=other)
        lat2.step(fa, fb, 2)
        ms = _time_steps(torch, lambda: lat2.step(fa, fb, steps), 1) / steps
        lat2.sync()
        rec = {"ms_per_step": round(ms, 4), "mlups": round(lat.n_nodes / (ms / 1e3) / 1e6, 2),
               "hbm_frac": round(8.0 * lat.Q * lat.n_nodes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        if other == "split_bf16x3":
            rec.update(mfma_record(lat2, ms))
        out[other] = rec
        lat2.close()
        _progress(f"{other}: {ms:.3f} ms/step")
    # additive collision f* = g + R (a' - a): the pulled populations are read twice (12 Q B/node)
    lat3 = Lattice(ab, deg, N, tau, [dict(nx=edge, ny=edge, nz=edge, bc_x=0)], precision="fp64_contract",
                   regularized=False)
    lat3.step(fa, fb, 2)
    ms = _time_steps(torch, lambda: lat3.step(fa, fb, steps), 1) / steps
    lat3.sync()
    lat3.close()
    out["additive_collision"] = {"ms_per_step": round(ms, 4), "mlups": round(lat.n_nodes / (ms / 1e3) / 1e6, 2),
                                 "bytes_per_launch": 12.0 * lat.Q * lat.n_nodes,
                                 "achieved_GBs": round(12.0 * lat.Q * lat.n_nodes / (ms / 1e3) / 1e9, 1)}
    _progress(f"additive collision: {ms:.3f} ms/step")
    lam_a, lam_b = lat.new_state(), lat.new_state()
    lam_a.normal_()
    dtau = torch.zeros(18, dtype=torch.float64, device="cuda")
    lat.step_adjoint(fa, lam_a, lam_b, dtau)
    ms_adj = _time_steps(torch, lambda: adjoint_pair(lat, fa, lam_a, lam_b, dtau), max(2, steps // 2)) / 2
    lat.sync()
    assert torch.isfinite(dtau).all()
    _progress(f"adjoint: {ms_adj:.3f} ms/step ({ms_adj / ms_fwd:.2f}x forward)")
    out["adjoint"] = {"ms_per_step": round(ms_adj, 4), "ratio_to_forward": round(ms_adj / ms_fwd, 3),
                      "reverse_sweep_ratio_with_replay": round((ms_adj + ms_fwd) / ms_fwd, 3),
                      "bytes_per_launch": 12.0 * lat.Q * lat.n_nodes,
                      "achieved_GBs": round(12.0 * lat.Q * lat.n_nodes / (ms_adj / 1e3) / 1e9, 1)}
    del lam_a, lam_b
    return out


CONTRACTION_TEXT = {"fp64_contract": "FP64 folded contractions", "fp32": "FP32 contractions",
                    "split_bf16x3": "split-BF16x3 matrix-core contractions"}


def step_kernel_name(lat, precision):
    if precision == "split_bf16x3":
        return f"k_collide_stream_bf16x3<{lat.Q1},{lat.N},false>"
    return f"k_collide_stream<{lat.Q1},{lat.N},false,{2 if precision == 'fp64_contract' else 0},1,false>"


def mfma_flops(lat):
    """Matrix-core flops per node-step of the split-BF16x3 form, three bf16 products each:
    algorithmic (projection of the orders 2..N, (M - 4) x Q, and the rebuild with its five
    correction columns, Q x (M + 5)) and issued (the same contractions padded to the 32 x 32 x 16
    tiles of v_mfma_f32_32x32x16_bf16: 32-row tiles of projected moments over ceil(Q1 / 2) or 6
    k-steps per x-slab, 32-row tiles of populations over 16-wide steps of the rebuild k axis)."""
    Q1, Q, M = lat.Q1, lat.Q, lat.M
    algorithmic = 2 * 3 * ((M - 4) * Q + Q * (M + 5))
    kpx = (Q1 + 1) // 2 if Q1 <= 8 else 6
    issued = 2 * 3 * (32 * math.ceil((M - 4) / 32) * Q1 * kpx * 16
                      + 32 * math.ceil(Q / 32) * 16 * math.ceil((M + 5) / 16))
    return algorithmic, issued


def mfma_record(lat, ms):
    alg, issued = mfma_flops(lat)
    n = lat.n_nodes
    return {"mfma_flops_per_node": alg, "mfma_issued_flops_per_node": issued,
            "mfma_TFLOPs": round(alg * n / (ms / 1e3) / 1e12, 1),
            "mfma_issued_TFLOPs": round(issued * n / (ms / 1e3) / 1e12, 1),
            "mfma_frac_of_bf16_peak": round(issued * n / (ms / 1e3) / 1e12 / MFMA_BF16_PEAK_TFLOPS, 4)}


def moment_state_bytes(lat):
    """Algorithmic HBM bytes per node of the three moment-state passes: z reads the M moment
    fields and writes the P2 (N+1) intermediate fields, y reads and writes P2 (N+1), x reads
    P2 (N+1) and writes M (FP32 each)."""
    n1 = (lat.N + 1) * (lat.N + 1) * (lat.N + 2) // 2
    return {"pass_z": 4.0 * (lat.M + n1), "pass_y": 8.0 * n1, "pass_x_collide": 4.0 * (n1 + lat.M)}


def time_moment_state(torch, lat, f_cur, f_other, steps, ms_pop):
    """The same step with the state held as the M moments (lbsmrt_step_moment_state): timed from
    the moments of the current population state, then one step of each form from that state,
    compared over every node.  Overwrites both population buffers with valid states."""
    ma = lat.project_state(f_cur)
    mb, work = lat.new_moment_state(), lat.new_moment_work()
    lat.step_moment_state(ma, mb, work, 2)
    lat.sync()
    ms = _time_steps(torch, lambda: lat.step_moment_state(ma, mb, work, 2), max(2, steps // 2)) / 2
    lat.sync()
    lat.project_state(f_cur, out=ma)
    lat.step(f_cur, f_other, 1)
    lat.step_moment_state(ma, mb, work, 1)
    lat.sync()
    lat.expand_state(mb, out=f_cur)
    worst = scale = 0.0
    for q0 in range(0, lat.Q, 49):
        worst = max(worst, float((f_cur[q0:q0 + 49] - f_other[q0:q0 + 49]).abs().max()))
        scale = max(scale, float(f_other[q0:q0 + 49].abs().max()))
    del ma, mb, work
    per = moment_state_bytes(lat)
    step_bytes = sum(per.values()) * lat.n_nodes
    out = {"ms_per_step": round(ms, 4), "mlups": round(lat.n_nodes / (ms / 1e3) / 1e6, 2),
           "speedup_vs_population_step": round(ms_pop / ms, 3),
           "bytes_per_node_step": {k: v for k, v in per.items()},
           "achieved_GBs_whole_step": round(step_bytes / (ms / 1e3) / 1e9, 1),
           "one_step_max_rel_diff_vs_population_step": worst / scale,
           "kernels": [f"k_ms_pass_z<{lat.Q1},{lat.N}>", f"k_ms_pass_y<{lat.Q1},{lat.N}>",
                       f"k_ms_pass_x_collide<{lat.Q1},{lat.N}>"]}
    _progress(f"moment-state step: {ms:.3f} ms ({out['mlups']} MLUPS, {ms_pop / ms:.2f}x the population step), "
              f"one-step difference {worst / scale:.2e}")
    return out


def time_shock_adjoint(torch, steps=300):
    """The adjoint-calibration shock (Ma 3, Nx 600, D3Q729, N = 5, FP64 contractions): forward and
    adjoint step times on one small domain, where each wave's latency, not HBM, sets the time."""
    from paper_2401_11086_amd import Lattice, solve_quadrature
    from paper_2401_11086_amd.shocks import shock_domain
    ab, deg, N = [1, 2, 3, 5], 11, 5
    c_l, _ = solve_quadrature(ab, deg)
    d, f, _ = shock_domain(3.0, 600, c_l)
    tau = {k: v for k, v in TAU_STAR.items() if k[0] <= N}
    lat = Lattice(ab, deg, N, tau, [d], shift_k=(2, 0, 0), precision="fp64_contract")
    fa = lat.equilibrium(torch.tensor(f, dtype=torch.float64, device="cuda"))
    fb = lat.new_state()
    lat.step(fa, fb, 10)
    ms_fwd = _time_steps(torch, lambda: lat.step(fa, fb, steps), 1) / steps
    ma, mb, work = lat.project_state(fa), lat.new_moment_state(), lat.new_moment_work()
    lat.step_moment_state(ma, mb, work, 10)
    ms_mom = _time_steps(torch, lambda: lat.step_moment_state(ma, mb, work, steps), 1) / steps
    lam_a, lam_b = lat.new_state(), lat.new_state()
    lam_a.normal_()
    dtau = torch.zeros(18, dtype=torch.float64, device="cuda")
    lat.step_adjoint(fa, lam_a, lam_b, dtau)
    ms_adj = _time_steps(torch, lambda: adjoint_pair(lat, fa, lam_a, lam_b, dtau), steps // 2) / 2
    lat.sync()
    assert torch.isfinite(dtau).all()
    lat.close()
    lat_b = Lattice(ab, deg, N, tau, [d], shift_k=(2, 0, 0), precision="split_bf16x3")
    ga, gb = lat_b.equilibrium(torch.tensor(f, dtype=torch.float64, device="cuda")), lat_b.new_state()
    lat_b.step(ga, gb, 10)
    ms_b = _time_steps(torch, lambda: lat_b.step(ga, gb, steps), 1) / steps
    lat_b.sync()
    lat_b.close()
    _progress(f"shock adjoint (Nx 600, D3Q729): forward {ms_fwd * 1e3:.1f} us (moment state {ms_mom * 1e3:.1f} us, "
              f"split-BF16x3 {ms_b * 1e3:.1f} us), adjoint {ms_adj * 1e3:.1f} us")
    return {"workload": "Ma 3 shock, Nx 600, D3Q729, N=5, FP64 contractions", "forward_us": round(ms_fwd * 1e3, 2),
            "forward_moment_state_us": round(ms_mom * 1e3, 2), "forward_split_bf16x3_us": round(ms_b * 1e3, 2),
            "adjoint_us": round(ms_adj * 1e3, 2), "ratio_to_forward": round(ms_adj / ms_fwd, 3)}


def time_shock_d3q4913(torch, steps=200):
    """Table 3's Ma 7 set D3Q4913 (D1Q17, degree 19, k = 3) on a 400-cell tube: the population
    step (eight lanes per node) against the moment-state step (sixteen lanes per node)."""
    from paper_2401_11086_amd import Lattice, solve_quadrature
    from paper_2401_11086_amd.shocks import shock_domain
    ab, deg, N = [1, 2, 3, 4, 5, 6, 7, 9], 19, 5
    c_l, _ = solve_quadrature(ab, deg)
    d, f, st = shock_domain(7.0, 400, c_l)
    tau = {k: v for k, v in TAU_STAR.items() if k[0] <= N}
    lat = Lattice(ab, deg, N, tau, [d], shift_k=(int(st["k"]), 0, 0), precision="fp64_contract")
    fa = lat.equilibrium(torch.tensor(f, dtype=torch.float64, device="cuda"))
    fb = lat.new_state()
    lat.step(fa, fb, 10)
    ms_pop = _time_steps(torch, lambda: lat.step(fa, fb, steps), 1) / steps
    ma, mb, work = lat.project_state(fa), lat.new_moment_state(), lat.new_moment_work()
    lat.step_moment_state(ma, mb, work, 10)
    ms_mom = _time_steps(torch, lambda: lat.step_moment_state(ma, mb, work, steps), 1) / steps
    lat.sync()
    launch = lat.launch_settings()
    lat.close()
    _progress(f"Ma 7 tube on D3Q4913 (400 cells): population {ms_pop * 1e3:.1f} us, moment state {ms_mom * 1e3:.1f} us")
    return {"workload": "Ma 7 shock, Nx 400, D3Q4913 (D1Q17 degree 19), N=5, FP64 contractions",
            "lanes_per_node_setting": launch["lanes_per_node"], "population_us": round(ms_pop * 1e3, 2),
            "moment_state_us": round(ms_mom * 1e3, 2), "speedup": round(ms_pop / ms_mom, 2)}


def time_batched(torch, n_shocks=64, steps=5000, seed=0):
    """Batched Mach sweep: n_shocks shocks with Ma ~ U[1.2, 5] and Nx ~ U{400..2000}, D3Q729
    (D1Q9 degree 11), N = 5, FP32 state, `steps` steps, in one context with the autotuned launch,
    against the same shocks stepped as separate contexts (one launch per shock per step)."""
    from paper_2401_11086_amd import Lattice, solve_quadrature
    from paper_2401_11086_amd import workloads as W
    from paper_2401_11086_amd.autotune import autotune, autotune_moment_state
    from paper_2401_11086_amd.shocks import shock_domain
    import numpy as np
    ab, deg, N = [1, 2, 3, 5], 11, 5
    c_l, _ = solve_quadrature(ab, deg)
    draws = W.mach_sweep(n_shocks, seed=seed)
    doms, fields = [], []
    for Ma, nx in draws:
        d, f, _ = shock_domain(Ma, nx, c_l)
        doms.append(d)
        fields.append(f)
    tau = {k: v for k, v in TAU_STAR.items() if k[0] <= N}
    lat = Lattice(ab, deg, N, tau, doms, shift_k=(2, 0, 0), precision="fp64_contract")
    fl = torch.tensor(np.concatenate(fields, axis=1), dtype=torch.float64, device="cuda")
    fa = lat.equilibrium(fl)
    fb = lat.new_state()
    f0 = fa.clone()
    tune = autotune(lat, fa, fb, steps=50, use_cache=False)
    fa.copy_(f0)
    ms = _time_steps(torch, lambda: lat.step(fa, fb, steps), 1) / steps
    lat.sync()
    nodes = lat.n_nodes
    out = {"workload": f"{n_shocks} shocks, Ma~U[1.2,5], Nx~U{{400..2000}} (sum {nodes}), D3Q729, N=5, "
                       f"{steps} steps", "nodes": nodes,
           "batched": {"launch": {"mode": tune["mode"], "block": tune["block"],
                                  "lanes_per_node": tune["lanes_per_node"]}, "ms_per_step": round(ms, 5),
                       "mlups": round(nodes / (ms / 1e3) / 1e6, 1),
                       "achieved_GBs": round(8.0 * lat.Q * nodes / (ms / 1e3) / 1e9, 1)},
           "autotune_trials": tune.get("trials")}
    _progress(f"batched sweep: {ms * 1e3:.1f} us/step ({tune['mode']}, {tune['block']}, "
              f"{tune['lanes_per_node']} lanes/node)")
    # the same batch with its state held as moments (line domains: the x-stage alone), with its
    # own autotuned launch (direct or captured, one or eight lanes per node)
    ma = lat.project_state(f0)
    mb = lat.new_moment_state()
    work = lat.new_moment_work()
    tune_m = autotune_moment_state(lat, ma, mb, work, steps=100, use_cache=False)
    lat.project_state(f0, out=ma)
    lat.step_moment_state(ma, mb, work, 2)
    lat.sync()
    ms_m = _time_steps(torch, lambda: lat.step_moment_state(ma, mb, work, steps), 1) / steps
    lat.sync()
    out["batched_moment_state"] = {"launch": {"mode": tune_m["mode"], "lanes_per_node": tune_m["lanes_per_node"]},
                                   "ms_per_step": round(ms_m, 5), "mlups": round(nodes / (ms_m / 1e3) / 1e6, 1),
                                   "bytes_per_node_step": 8.0 * lat.M,
                                   "speedup_vs_population_batch": round(ms / ms_m, 2),
                                   "autotune_trials": tune_m.get("trials")}
    _progress(f"batched sweep, moment state: {ms_m * 1e3:.1f} us/step ({tune_m['mode']}, "
              f"{tune_m['lanes_per_node']} lanes/node)")
    del ma, mb
    # the same batch with the split-BF16x3 matrix-core contractions (one launch per step)
    lat_b = Lattice(ab, deg, N, tau, doms, shift_k=(2, 0, 0), precision="split_bf16x3")
    ga, gb = lat_b.equilibrium(fl), lat_b.new_state()
    lat_b.step(ga, gb, 2)
    lat_b.sync()
    ms_b = _time_steps(torch, lambda: lat_b.step(ga, gb, steps), 1) / steps
    lat_b.sync()
    out["batched_split_bf16x3"] = {"ms_per_step": round(ms_b, 5), "mlups": round(nodes / (ms_b / 1e3) / 1e6, 1),
                                   "achieved_GBs": round(8.0 * lat.Q * nodes / (ms_b / 1e3) / 1e9, 1),
                                   "speedup_vs_population_batch": round(ms / ms_b, 3),
                                   **mfma_record(lat_b, ms_b)}
    _progress(f"batched sweep, split-BF16x3: {ms_b * 1e3:.1f} us/step")
    lat_b.close()
    del ga, gb
    # the same shocks as separate contexts, one launch per shock per step
    sep = []
    for d, f in zip(doms, fields):
        one = Lattice(ab, deg, N, tau, [d], shift_k=(2, 0, 0), precision="fp64_contract")
        ga = one.equilibrium(torch.tensor(f, dtype=torch.float64, device="cuda"))
        sep.append((one, ga, one.new_state()))
    torch.cuda.synchronize()

    def run_sep():
        for t in range(steps):
            for one, ga, gb in sep:
                one.step(ga, gb, 1) if t % 2 == 0 else one.step(gb, ga, 1)
    ms_sep = _time_steps(torch, run_sep, 1) / steps
    for one, _, _ in sep:
        one.sync()
    out["separate_contexts"] = {"ms_per_step": round(ms_sep, 5), "mlups": round(nodes / (ms_sep / 1e3) / 1e6, 1)}
    out["speedup_batched_vs_separate"] = round(ms_sep / ms, 2)
    _progress(f"separate contexts: {ms_sep * 1e3:.1f} us/step")
    # every context is destroyed here, while the runtime is up, not at interpreter teardown
    for one, _, _ in sep:
        one.close()
    sep.clear()
    lat.close()
    del fa, fb, f0, fl
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="box256_q343_n4", choices=sorted(WORKLOADS))
    ap.add_argument("--kn", type=float, default=0.05)
    ap.add_argument("--precision", default="fp64_contract", choices=list(PRECISIONS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-only", action="store_true", help="run only the batched Mach sweep")
    ap.add_argument("--batched-steps", type=int, default=5000)
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP32-contraction and adjoint timings")
    ap.add_argument("--variants", default="moment_state,forms,shock_adjoint,d3q4913,batched",
                    help="comma list of the variant groups to time after the main step: moment_state, forms "
                         "(other contraction forms, additive collision, adjoint), shock_adjoint, d3q4913, batched")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="time a plain device copy of one f buffer instead (HBM calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
                                   "described in DESIGN.md but not built)"}))
        sys.exit(2)

    import torch

    from paper_2401_11086_amd import Lattice
    from paper_2401_11086_amd import workloads as W

    ab, deg, N, edge = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    if args.batched_only:
        print(json.dumps({"batched_mach_sweep": time_batched(torch, steps=args.batched_steps)}), flush=True)
        return
    if args.calibrate_copy:
        copy_calibration(torch, 343 * edge ** 3 if N == 4 else 729 * edge ** 3, args.steps, args.warmup)
        return
    _progress(f"workload {args.workload} ({args.precision}): building lattice")
    r_guess = {9: 1.19697977039307, 11: 0.678003906334339}[deg]
    tau20 = args.kn * edge * r_guess
    tau = {k: v * tau20 for k, v in TAU_STAR.items() if k[0] <= N}
    lat = Lattice(ab, deg, N, tau, [dict(nx=edge, ny=edge, nz=edge, bc_x=0)], precision=args.precision)
    assert abs(lat.c_l - r_guess) < 1e-12
    fields = W.fourier_box_torch(edge, "cuda")
    fa = lat.equilibrium(fields)
    del fields
    fb = lat.new_state()
    torch.cuda.synchronize()
    _progress(f"state ready: 2 x {fa.numel() * 4 / 1e9:.1f} GB; warmup {args.warmup}")
    cur = lat.step(fa, fb, args.warmup) if args.warmup > 0 else fa
    if cur is fb:
        fa, fb = fb, fa
    lat.sync()
    _progress(f"timing {args.steps} steps")
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    cur = lat.step(fa, fb, args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat.sync()
    gpu_ms = ev0.elapsed_time(ev1)
    ms_step = gpu_ms / args.steps
    nodes = lat.n_nodes
    mlups = nodes * args.steps / (gpu_ms / 1e3) / 1e6
    bytes_per_launch = 8.0 * lat.Q * nodes
    achieved = bytes_per_launch / (ms_step / 1e3) / 1e9
    _progress(f"{ms_step:.3f} ms/step, {mlups:.1f} MLUPS, {achieved:.0f} GB/s (wall {wall:.2f} s)")
    rho = lat.moments(cur)[0]
    assert torch.isfinite(rho).all() and abs(float(rho.mean()) - 1.0) < 1e-3
    variants = {}
    groups = set() if args.no_variants else {g.strip() for g in args.variants.split(",") if g.strip()}
    if "moment_state" in groups:
        variants["moment_state"] = time_moment_state(torch, lat, cur, fb if cur is fa else fa, args.steps, ms_step)
    if "forms" in groups:
        variants.update(time_variants(torch, lat, fa, fb, ab, deg, N, tau, edge, args, ms_step))
    if "shock_adjoint" in groups:
        variants["shock_adjoint"] = time_shock_adjoint(torch)
    if "d3q4913" in groups:
        variants["shock_d3q4913"] = time_shock_d3q4913(torch)
    if "batched" in groups:
        variants["batched_mach_sweep"] = time_batched(torch, steps=args.batched_steps)

    out = {
        "metric": "MLUPS & % HBM/MFMA roofline, SMRT collide-stream; FP32 vs split-BF16; adjoint",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # arithmetic type of the contractions (the state is stored in FP32 in every form)
        "dtype": {"fp64_contract": "f64", "fp32": "f32", "split_bf16x3": "bf16x3"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{edge}^3 periodic box, D3Q{lat.Q} (D1Q{lat.Q1} degree {deg}), Hermite N={N}, "
                               f"Kn={args.kn}, 16 Fourier modes per field, FP32 state, "
                               + CONTRACTION_TEXT[args.precision] + ", FP64 moment section",
                   "nodes": nodes, "Q": lat.Q, "M": lat.M, "precision": args.precision},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": recorded_traffic(args.workload, args.precision),
                     "kernel": step_kernel_name(lat, args.precision),
                     "bytes_per_launch": bytes_per_launch},
    }
    if args.precision == "split_bf16x3":
        # the matrix-core roofline of the same launch (algorithmic bf16 flops)
        mf = mfma_record(lat, ms_step)
        out["roofline_mfma"] = {"bound": "mfma", "achieved": mf["mfma_TFLOPs"], "peak": MFMA_BF16_PEAK_TFLOPS,
                                "unit": "TFLOP/s", "frac": round(mf["mfma_TFLOPs"] / MFMA_BF16_PEAK_TFLOPS, 4),
                                **mf}
    if variants:
        out["variants"] = variants
    # measured streaming ceiling on the same buffers (a plain copy, read + write)
    ceiling = copy_ceiling(torch, fa, fb)
    out["roofline"]["copy_GBs_same_buffers"] = round(ceiling, 1)
    out["roofline"]["frac_of_copy"] = round(achieved / ceiling, 4)
    _progress(f"device copy of one state buffer: {ceiling:.0f} GB/s; step kernel at {achieved / ceiling:.2f} of it")
    if not args.no_cpu_baseline:
        _progress("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(torch, ab, deg, N, edge, args.kn)
        _progress("oracle and GPU on two shock tubes")
        out["cpu_baseline"]["shock_samples"] = shock_samples(torch)
    out["device"] = device_record(torch)
    lat.close()
    del fa, fb, cur
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
