"""Benchmark: spring-steps/s of the HIP mass-spring step on one MI355X, with its HBM roofline
fraction and the FP64 oracle timed on the host as a reported CPU baseline.

Workload (default): the cantilever beam of 400 x 40 x 40 nodes (640,000 masses, 8,020,476
springs, 0.005 m spacing, per-voxel stiffness for E = 1 MPa, one end face fixed, gravity on,
no ground, dt = 5e-5 s), synthetic and seeded.  One step = one time step of the whole body.
``--workload population``: 1024 random-walk robots (node targets log-uniform in [500, 50k],
3 materials, 32 actuation groups each, contact plane, dt = 1e-4 s) stepped together, one
launch per step; also reports rollouts/s for the 5000-step rollout.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--workload W] [--tune]

Prints ONE JSON line.  Timing: W untimed steps, then exactly K steps bracketed by
torch.cuda.synchronize() and HIP events recorded on the stream the library launches on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spring-steps/sec + % HBM roofline; surrogate vs plain sim evals/sec"
HBM_PEAK_GBS = 8000.0
VALU_PEAK = 256 * 2.4e9          # wave64 VALU instructions per second: 256 CUs x 2.4 GHz x 1 per CU

# Issue cycles of the method's arithmetic per incidence (one spring seen from one end), in the
# FP64-numerator formulation every step form shares: 19 full-rate VALU instructions (3
# differences, 3 widenings to FP64, an FP64 multiply and 2 FMAs for |d|^2, the FP64 subtraction
# of L0^2, 2 narrowings, the denominator FMA and floor, 2 multiplies, 3 FMAs into the force) and
# 2 quarter-rate ones (sqrt, reciprocal) at 4 cycles; an actuated spring adds 3 (L0 times its
# factor, widening, squaring).  Per wave64 instruction: 64 incidences.
ALU_CYCLES_PER_INCIDENCE = 19 + 2 * 4
ALU_CYCLES_ACTUATED = 3


def alu_cycles(n_springs: int, actuated: bool = False) -> float:
    """Algorithmic VALU issue cycles of one step (all CUs together): 2 incidences per spring."""
    return 2.0 * n_springs * (ALU_CYCLES_PER_INCIDENCE + (ALU_CYCLES_ACTUATED if actuated else 0)) / 64.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_grid_kernel_cantilever_400x40x40.traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2207_09334_amd", "csrc", "kernels.hip")


def formula_bytes(n_masses: int, n_springs: int, actuated: bool = False, batched: bool = False) -> int:
    """HBM traffic of one step of a per-mass CSR method with explicit incidences: per mass
    read x, v and write x, v (48 B), 1/m (4 B), a row offset (4 B); per spring two incidences
    of (neighbour, k, L0) = 24 B; +2 B per spring when actuated, +4 B per mass when batched.
    The step kernel's own encodings move less (see kernel_bytes)."""
    b = 56 * n_masses + 24 * n_springs
    if actuated:
        b += 2 * n_springs
    if batched:
        b += 4 * n_masses
    return b


# bytes per incidence of each step form's entry stream: 16-bit words (neighbour slot and
# (k, L0) pair index), 32-bit words, explicit (16-bit slot + FP32 k and L0; + a 16-bit
# factor index when actuated), split (32-bit entry + a 4-byte record per spring end held)
ENTRY_BYTES = {"narrow": 2, "table": 4, "explicit": 10, "split": 6, "resident": 4, "grid": 0}


def kernel_bytes(n_masses: int, n_springs: int, form: str, actuated: bool = False) -> int:
    """Compulsory HBM bytes of one launch of the step kernel in its entry encoding: per mass
    read and write x (float4: position and 1/m, 16 + 16 B) and v (12 + 12 B) and the lane's
    2-byte mass index (58 B); per spring its two incidence entries.  The structured-box form
    reads no incidence data and no lane map (56 B per mass).  Slice padding, halo re-reads,
    halo lists and the parameter table are overhead, not counted."""
    per_inc = ENTRY_BYTES[form] + (2 if actuated and form == "explicit" else 0)
    if form == "grid":   # no incidence data and no lane map: the state alone
        return 56 * n_masses
    return 58 * n_masses + 2 * per_inc * n_springs


def kernel_source_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()


def profile_record(workload: str, launch: dict):
    """The committed rocprofv3 counter summary of the step kernel (HBM bytes and VALU
    instructions per launch), or None when it was taken for another workload or launch
    configuration, or before the kernel source last changed."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernels_sha256") != kernel_source_hash() or rec.get("workload") != workload:
        return None
    if any(rec.get(k) != launch.get(k) for k in ("block_masses", "batch", "persistent_groups", "step_form")):
        return None
    if rec.get("lanes_per_mass", 1) != launch.get("lanes_per_mass", 1):
        return None
    return rec


def cpu_baseline(workload, steps: int):
    import numpy as np

    from oracle import lattice as L
    from oracle import physics as P

    if len(workload.bodies) > 8:      # a bounded sample: the first 8 robots of the population
        import dataclasses
        G = workload.n_groups
        workload = dataclasses.replace(workload, name=workload.name + "[first 8 robots]",
                                       bodies=workload.bodies[:8], phase=workload.phase[:8 * G],
                                       amp=workload.amp[:8 * G])
    lat = L.build(workload)
    sys_ = P.system_from(lat, workload)
    x, v = lat.x.copy(), np.zeros_like(lat.x)
    from threadpoolctl import threadpool_limits

    with threadpool_limits(limits=1):     # one thread, also for any BLAS call NumPy makes
        x, v = P.step(sys_, x, v, 0)      # untimed first step (page-in)
        t0 = time.perf_counter()
        x, v = P.run(sys_, x, v, 1, steps)
        dt = time.perf_counter() - t0
    return {"value": lat.n_springs * steps / dt, "unit": "spring-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} FP64 NumPy steps of the full {workload.name} lattice "
                      f"({lat.n_masses} masses, {lat.n_springs} springs), single thread on {cpu_model()} "
                      f"({len(os.sched_getaffinity(0))} cores available), {dt:.1f} s"}


def _cpu_worker(workload, steps, barrier, out):
    """One process of the all-cores baseline: builds the oracle's lattice, takes one untimed
    step, waits for the others, then times `steps` single-threaded steps."""
    os.environ["OMP_NUM_THREADS"] = "1"
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import lattice as L
    from oracle import physics as P

    lat = L.build(workload)
    sys_ = P.system_from(lat, workload)
    x, v = lat.x.copy(), np.zeros_like(lat.x)
    with threadpool_limits(limits=1):
        x, v = P.step(sys_, x, v, 0)
        barrier.wait()
        t0 = time.time()
        x, v = P.run(sys_, x, v, 1, steps)
        t1 = time.time()
    out.put((t0, t1, lat.n_springs * steps))


def cpu_baseline_all_cores(workload, steps: int, procs: int):
    """The oracle on every host core at once: `procs` processes (started fresh, not forked
    from this GPU process), each stepping its own copy of the workload single-threaded, all
    timed over the same window; rate = all their spring-steps / (last end - first start)."""
    import multiprocessing as mp

    ctx = mp.get_context("spawn")
    barrier, out = ctx.Barrier(procs), ctx.Queue()
    ps = [ctx.Process(target=_cpu_worker, args=(workload, steps, barrier, out)) for _ in range(procs)]
    for p in ps:
        p.start()
    res = [out.get() for _ in ps]
    for p in ps:
        p.join()
    t0, t1 = min(r[0] for r in res), max(r[1] for r in res)
    work = sum(r[2] for r in res)
    return {"value": work / (t1 - t0), "unit": "spring-steps/s", "cores": procs, "kind": "oracle",
            "sample": f"{procs} processes, each {steps} FP64 NumPy steps of its own copy of the full {workload.name} "
                      f"lattice, single-threaded, on {cpu_model()}; {t1 - t0:.1f} s window"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def adjoint_bench(args) -> dict:
    """Gait gradient of the actuated quadruped: forward rollout of 2000 steps keeping a
    checkpoint every 100 steps, then the adjoint (segments recomputed from the checkpoints),
    against the plain forward rollout on HIP graphs."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2207_09334_amd import autograd as AG
    from paper_2207_09334_amd import cronos as CR
    from paper_2207_09334_amd import problem as PR

    w = W.quadruped()
    stream = torch.cuda.Stream()
    # the launch shape (workgroup size, batch, lanes per mass) from the autotuner unless given
    tune = 0 if (args.block or args.lanes) else 20
    sim, lat, x0 = PR.create(w, stream=stream.cuda_stream, block_masses=args.block, lanes_per_mass=args.lanes,
                             tune_steps=tune)
    v0 = np.zeros_like(x0)
    lw = AG.forward_displacement_weights(lat.mass)
    T, K = args.adjoint_steps, 100
    ph, am = np.asarray(w.phase, float), np.asarray(w.amp, float)

    def plain():
        CR.cronos_set_state(sim, x0, v0, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        CR.cronos_step(sim, T)
        CR.cronos_read_state(sim)                 # blocks until the rollout is done
        return time.perf_counter() - t0

    def grad():
        CR.cronos_set_state(sim, x0, v0, 0)
        CR.cronos_set_actuation(sim, ph, am, w.freq_hz)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = CR.cronos_rollout(sim, T, K, lw)
        t1 = time.perf_counter()
        dp, da = CR.cronos_rollout_backward(sim)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, loss, dp, da

    CR.cronos_set_actuation(sim, ph, am, w.freq_hz)
    plain()
    first = grad()                                # warm-up: allocations, the sweep's graph capture
    t_plain = min(plain() for _ in range(3))
    runs = [grad() for _ in range(3)]
    t_fwd = min(r[0] for r in runs)
    t_bwd = min(r[1] for r in runs)
    _, _, loss, dp, da = runs[-1]
    repeat = all(np.array_equal(r[3], dp) and np.array_equal(r[4], da) for r in runs)
    return {
        "metric": "adjoint gait gradient: gradients/s (forward with checkpoints + backward)",
        "value": 1.0 / (t_fwd + t_bwd), "unit": "gradients/s", "higher_is_better": True, "dtype": "f32 (FP64 parameter sums)",
        "data": "synthetic",
        "config": {"workload": w.name, "n_masses": int(lat.n_masses), "n_springs": int(len(lat.ends)),
                   "steps": T, "checkpoint_every": K, "parameters": int(2 * len(ph)),
                   "block_masses": CR.cronos_launch_config(sim)["block_masses"],
                   "lanes_per_mass": CR.cronos_launch_config(sim)["lanes_per_mass"],
                   "batch": CR.cronos_launch_config(sim)["batch"], "autotuned": bool(tune)},
        "forward_with_checkpoints_s": t_fwd, "backward_s": t_bwd, "plain_forward_s": t_plain,
        "first_backward_s": first[1],
        "gradient_over_plain_forward": (t_fwd + t_bwd) / t_plain, "loss": loss,
        "bitwise_repeatable": bool(repeat),
    }


def frequency_bench(args) -> dict:
    """Natural frequency at GPU scale (sections "Euler-Bernoulli Beam Tests" and "Natural
    Frequency Analysis"): cantilevers of several lengths, widths and heights start bent
    along the clamped-free beam's first mode shape (tip amplitude L / 2000 in z, no gravity,
    no damping) and oscillate freely.  As in the paper, the frequency comes from a Fourier
    transform of the tracked motion: the FP64 centre-of-mass height, sampled 200 times per
    expected period over 6.4 periods, Hann-windowed, its spectral peak refined by parabolic
    interpolation; it is compared with K^2/(2 pi) sqrt(E I / (rho A L^4)), K = 1.8751."""
    import math

    import numpy as np
    import torch

    import workloads as W
    from paper_2207_09334_amd import cronos as CR
    from paper_2207_09334_amd import problem as PR

    K1, E, rho, a = 1.8751040687, 1.0e6, 1000.0, 0.005
    rows, t_sim, steps_total = [], 0.0, 0
    for nx, ny, nz in args.sweep:
        w = W.cantilever(nx, ny, nz, youngs=E, spacing=a)
        Lb, Wd, H = (nx - 1) * a, (ny - 1) * a, (nz - 1) * a
        f_eb = K1 ** 2 / (2 * math.pi) * math.sqrt(E * (Wd * H ** 3 / 12.0) / (rho * Wd * H * Lb ** 4))
        stream = torch.cuda.Stream()
        lat = PR.build_lattice(w)
        x0 = PR.initial_positions(w, lat).copy()
        # first clamped-free mode: cosh(bx) - cos(bx) - s (sinh(bx) - sin(bx)), b = K / L
        bx = K1 * (x0[:, 0] - x0[:, 0].min()) / Lb
        sg = (math.cosh(K1) + math.cos(K1)) / (math.sinh(K1) + math.sin(K1))
        phi = np.cosh(bx) - np.cos(bx) - sg * (np.sinh(bx) - np.sin(bx))
        x0[:, 2] += (Lb / 2000.0) * phi / np.abs(phi).max()
        sim, lat, _ = PR.create(w, lat=lat, x0=x0, stream=stream.cuda_stream, gravity=(0.0, 0.0, 0.0))
        every = max(16, int(round(1.0 / f_eb / w.dt / 200 / 16)) * 16)
        n_samples = int(6.4 * 200)
        z = np.empty(n_samples + 1)
        z[0] = CR.cronos_diagnostics(sim)[0]["com"][2]
        t0 = time.perf_counter()
        for q in range(1, n_samples + 1):
            CR.cronos_step(sim, every)
            z[q] = CR.cronos_diagnostics(sim)[0]["com"][2]
        t_sim += time.perf_counter() - t0
        steps_total += n_samples * every
        f_sim = spectral_peak(z, every * w.dt)
        info = CR.cronos_info(sim)
        rows.append({"nodes": [nx, ny, nz], "masses": info["n_masses"], "springs": info["n_springs"],
                     "L_m": Lb, "W_m": Wd, "H_m": H, "f_sim_hz": f_sim, "f_euler_bernoulli_hz": f_eb,
                     "ratio": f_sim / f_eb, "steps": n_samples * every})
        sim.close()
        print(f"frequency: {nx}x{ny}x{nz} f_sim {f_sim:.4f} Hz, EB {f_eb:.4f} Hz", file=sys.stderr, flush=True)
    # static tip deflection of the 400 x 40 x 40 beam under a small load (tip deflection L/1000),
    # relaxed with velocity damping that critically damps the first mode, against w L^4 / (8 E I)
    w = W.cantilever(400, 40, 40, youngs=E, spacing=a)
    Lb, H = 399 * a, 39 * a
    g = 1e-3 * Lb * E * H ** 2 / (1.5 * rho * Lb ** 4)
    w1 = K1 ** 2 * math.sqrt(E * H ** 2 / 12.0 / (rho * Lb ** 4))
    stream = torch.cuda.Stream()
    sim, lat, x0 = PR.create(w, stream=stream.cuda_stream, gravity=(0.0, 0.0, -g), damping=2.0 * w1 * w.dt)
    tip = lat.coords[:, 0] == lat.coords[:, 0].max()
    t0 = time.perf_counter()
    CR.cronos_step(sim, int(round(6.0 / w.dt)))
    xg, _, _ = CR.cronos_read_state(sim)
    t_defl = time.perf_counter() - t0
    sim.close()
    defl = float(-(xg[tip, 2] - x0[tip, 2]).mean())
    d_eb = 1.5 * rho * g * Lb ** 4 / (E * H ** 2)
    deflection = {"nodes": [400, 40, 40], "g_eff": g, "tip_deflection_m": defl, "euler_bernoulli_m": d_eb,
                  "ratio": defl / d_eb, "steps": int(round(6.0 / w.dt)), "seconds": t_defl}
    print(f"frequency: 400x40x40 tip deflection {defl:.4e} m, EB {d_eb:.4e} m", file=sys.stderr, flush=True)
    return {"metric": "simulated / Euler-Bernoulli first frequency", "value": float(np.mean([r["ratio"] for r in rows])),
            "unit": "ratio", "higher_is_better": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "cantilever_sweep", "youngs": E, "density": rho, "spacing": a},
            "beams": rows, "sim_seconds": t_sim, "steps": steps_total, "tip_deflection": deflection}


def modes_bench(args) -> dict:
    """Natural frequencies by the device's Lanczos solver (section "Natural Frequency
    Analysis": the generalised eigenproblem of the linearised system) for the cantilevers of
    the frequency sweep at rest: the two lowest distinct frequencies, the Lanczos steps they
    took and the time, compared with the two lowest distinct Euler-Bernoulli frequencies of
    bending in either plane (first and second clamped-free roots K = 1.8751, 4.6941)."""
    import math

    import numpy as np
    import torch

    import workloads as W
    from paper_2207_09334_amd import cronos as CR
    from paper_2207_09334_amd import problem as PR

    K1, E, rho, a = 1.8751040687, 1.0e6, 1000.0, 0.005
    rows, t_all = [], 0.0
    for nx, ny, nz in args.sweep:
        w = W.cantilever(nx, ny, nz, youngs=E, spacing=a)
        Lb, Wd, H = (nx - 1) * a, (ny - 1) * a, (nz - 1) * a
        eb = sorted(Kr ** 2 / (2 * math.pi) * math.sqrt(E * D * D / 12.0 / (rho * Lb ** 4))
                    for Kr in (K1, 4.6940911330) for D in (H, Wd))
        eb = [f for q, f in enumerate(eb) if q == 0 or f > eb[q - 1] * (1 + 1e-9)][:2]
        stream = torch.cuda.Stream()
        sim, _, _ = PR.create(w, stream=stream.cuda_stream, gravity=(0.0, 0.0, 0.0))
        t0 = time.perf_counter()
        om, iters = CR.cronos_natural_frequencies(sim, n_modes=2, max_iter=args.modes_iter, tol=1e-9)
        dt = time.perf_counter() - t0
        t_all += dt
        info = CR.cronos_info(sim)
        f = [float(o / (2 * math.pi)) for o in om]
        rows.append({"nodes": [nx, ny, nz], "masses": info["n_masses"], "springs": info["n_springs"],
                     "f_hz": f, "f_euler_bernoulli_hz": eb, "ratio": [fq / e for fq, e in zip(f, eb)],
                     "lanczos_steps": iters, "seconds": dt, "us_per_step": 1e6 * dt / max(iters, 1)})
        sim.close()
        print(f"modes: {nx}x{ny}x{nz} f {f} Hz (EB {eb}), {iters} steps, {dt:.2f} s", file=sys.stderr, flush=True)
    return {"metric": "Lanczos first frequency / Euler-Bernoulli",
            "value": float(np.mean([r["ratio"][0] for r in rows if r["ratio"]])),
            "unit": "ratio", "higher_is_better": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "cantilever_modes", "youngs": E, "density": rho, "spacing": a},
            "beams": rows, "seconds": t_all}


def spectral_peak(z, h: float) -> float:
    """Frequency (Hz) of the strongest component of samples z taken every h seconds: mean
    removed, Hann window, zero-padded FFT, peak refined by a parabola through the log
    magnitudes of its bin and the two beside it."""
    import numpy as np

    s = np.asarray(z, dtype=np.float64)
    s = (s - s.mean()) * np.hanning(len(s))
    n = 8 * len(s)
    mag = np.abs(np.fft.rfft(s, n))
    k = int(np.argmax(mag[1:-1])) + 1
    la, lb, lc = np.log(mag[k - 1:k + 2] + 1e-300)
    off = 0.5 * (la - lc) / (la - 2.0 * lb + lc) if la - 2.0 * lb + lc != 0.0 else 0.0
    return (k + off) / (n * h)


MFMA_BF16_PEAK_TFLOPS = 2500.0   # dense BF16 matrix-core peak of the MI355X


def mlp_flops(sizes, rows: int) -> float:
    """Matrix-product flops of one training step of the perceptron over `rows` rows: forward
    Z = H W (2 rows K N per layer), weight gradient H^T dZ (the same) and back-propagation
    dZ W^T (the same, except into the first layer's input)."""
    per = [2.0 * rows * sizes[l] * sizes[l + 1] for l in range(len(sizes) - 1)]
    return 3.0 * sum(per) - per[0]


def mlp_bench(args) -> dict:
    """Surrogate network training throughput on synthetic data of the surrogate's shapes: 96
    inputs, three hidden layers of `width`, 3 outputs, minibatches of 1024 rows, `epochs`
    epochs over `mlp_rows` rows; the matrix-product rate against the BF16 MFMA peak."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2207_09334_amd import cronos as CR

    sizes = (96, args.width, args.width, args.width, 3)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(args.mlp_rows, sizes[0])).astype(np.float32)
    T = np.tanh(X[:, :3] + 0.1 * X[:, 3:6] * X[:, 6:9]).astype(np.float32)
    batch = 1024
    net = CR.cronos_mlp_create(W.mlp_init(4, sizes), max_rows=batch)
    CR.cronos_mlp_train(net, X[:batch * 4], T[:batch * 4], batch=batch, epochs=1, lr=1e-3, seed=1)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = CR.cronos_mlp_train(net, X, T, batch=batch, epochs=args.epochs, lr=1e-3, seed=2)
    sec = time.perf_counter() - t0
    steps = args.epochs * ((args.mlp_rows + batch - 1) // batch)
    flops = args.epochs * mlp_flops(sizes, args.mlp_rows)
    xf = rng.normal(size=(65536, sizes[0])).astype(np.float32)
    CR.cronos_mlp_forward(net, xf[:batch])
    t1 = time.perf_counter()
    CR.cronos_mlp_forward(net, xf)
    fsec = time.perf_counter() - t1
    tf = flops / sec / 1e12
    return {"metric": "surrogate MLP training matrix-product rate", "value": tf, "unit": "TFLOP/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "bf16", "data": "synthetic",
            "config": {"workload": f"mlp_96x{args.width}x{args.width}x{args.width}x3", "rows": args.mlp_rows,
                       "batch": batch, "epochs": args.epochs},
            "roofline": {"bound": "mfma", "achieved": tf, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / MFMA_BF16_PEAK_TFLOPS},
            "train_seconds": sec, "us_per_minibatch": sec / steps * 1e6, "last_epoch_loss": loss,
            "forward_rows_per_s": len(xf) / fsec}


def surrogate_bench(args) -> dict:
    """Surrogate screening vs the plain batched simulator.  Morphology pools of `pool` robots
    (seed 4, disjoint robot-index ranges) are each simulated under `draws` actuation draws
    (5000 steps each); the robots of the first `pools` pools train the network, those of the
    next `held_pools` pools are held-out candidates scored by the simulator."""
    import numpy as np

    from paper_2207_09334_amd import cronos as CR
    from paper_2207_09334_amd import surrogate as SG

    G = 32
    Xtr, Dtr, Xte, Dte = [], [], [], []
    held_bodies, ph_c, am_c, body_of = [], [], [], []
    sim_seconds, rollouts, noise_floor, noise_floor_x = 0.0, 0, None, None
    material_k = spacing = None
    for p in range(args.pools + args.held_pools):
        pool = SG.Pool(args.pool, seed=4, steps=5000, first_robot=p * args.pool)
        material_k, spacing = pool.workload.material_k, pool.workload.spacing
        held = p >= args.pools
        for d in range(args.draws):
            X, D = pool.draw(d)
            (Xte if held else Xtr).append(X)
            (Dte if held else Dtr).append(D)
            if held:
                ph, am = pool.actuation(d)
                ph_c.append(ph)
                am_c.append(am)
                body_of.append(np.arange(args.pool, dtype=np.int32) + len(held_bodies))
        if p == 0:
            # the simulator's own noise floor on this target: draw 0 again with every phase
            # moved by 1e-6 rad; the chaotic part of the displacement is beyond any predictor
            ph0, am0 = pool.actuation(0)
            Dp = pool.rollout(ph0 + 1e-6, am0)
            noise_floor = SG.rms_relative_error(Dp, Dtr[0])
            # the same for the forward (x) component alone: how much of it the dynamics decide
            # beyond what any predictor of the inputs could know
            noise_floor_x = float(np.sqrt(((Dp[:, 0] - Dtr[0][:, 0]) ** 2).mean() / (Dtr[0][:, 0] ** 2).mean()))
        if held:
            held_bodies.extend(pool.workload.bodies)
        sim_seconds += pool.sim_seconds
        rollouts += pool.rollouts_done
        pool.close()
        print(f"surrogate: pool {p} done ({'held-out' if held else 'training'})", file=sys.stderr, flush=True)
    sim_rate = rollouts / sim_seconds
    if args.dump:
        # the data set in compact form: features and displacements per (pool, draw, robot)
        os.makedirs(args.dump, exist_ok=True)
        # (the actuation columns follow from workloads.population_actuation per pool and draw)
        per = args.draws
        morph_tr = np.concatenate([Xtr[p * per][:, :32] for p in range(args.pools)])
        morph_te = np.concatenate([Xte[p * per][:, :32] for p in range(args.held_pools)])
        np.savez_compressed(os.path.join(args.dump, "surrogate_data.npz"), morph_train=morph_tr,
                            D_train=np.concatenate(Dtr), morph_held=morph_te, D_held=np.concatenate(Dte),
                            pool=args.pool, pools=args.pools, held_pools=args.held_pools, draws=args.draws)
    Xtr, Dtr, Dte = np.concatenate(Xtr), np.concatenate(Dtr), np.concatenate(Dte)
    sur = SG.Surrogate(Xtr, Dtr, epochs=args.epochs, batch=1024, width=args.width, lr=args.lr,
                       lr_final=args.lr_final if args.lr_final >= 0 else None)
    # screening throughput: candidates are (robot, actuation) pairs; the robots' morphology
    # descriptors are computed once, each candidate's features assembled natively, then predicted
    body_of = np.concatenate(body_of)
    ph_c, am_c = np.concatenate(ph_c), np.concatenate(am_c)
    # per-robot work (morphology descriptors; for the simulator: lattice, layout, upload) is
    # left out of both rates; per-candidate work is in both (simulator: the rollout)
    # (the screening pass is a few milliseconds: it is timed three times and the fastest kept,
    # the simulator's rate being a steady rate over all its rollouts)
    t0 = time.perf_counter()
    morph = CR.cronos_features(held_bodies, material_k, spacing, 0, None, None)
    t_morph = time.perf_counter() - t0
    t_screen = []
    for _ in range(3):
        t1 = time.perf_counter()
        Xc = CR.cronos_candidate_features(body_of, morph, G, ph_c, am_c)
        pred = sur.predict(Xc)
        flagged = sur.out_of_distribution(Xc)
        t_screen.append(time.perf_counter() - t1)
    n_cand = len(Xc)
    sur_rate = n_cand / min(t_screen)
    sur_rate_morph = n_cand / (min(t_screen) + t_morph)
    err = SG.rms_relative_error(pred, Dte)
    per = np.linalg.norm(pred - Dte, axis=1) / np.sqrt((Dte ** 2).sum(axis=1).mean())
    k = max(1, n_cand // 20)
    chosen = SG.screen(pred, flagged, k)
    true_top = set(np.argsort(-Dte[:, 0], kind="stable")[:k].tolist())
    pred_top = set(np.argsort(-pred[:, 0], kind="stable")[:k].tolist())
    # baseline without the network: a constant (training-mean) prediction
    err_mean = SG.rms_relative_error(np.broadcast_to(Dtr.mean(axis=0), Dte.shape), Dte)
    return {
        "metric": "surrogate vs plain sim evals/sec", "value": sur_rate / sim_rate, "unit": "x",
        "higher_is_better": True, "dtype": "bf16 (MFMA, FP32 accumulation)", "data": "synthetic",
        "config": {"workload": f"surrogate_{args.pools}x{args.pool}robots_draws{args.draws}", "rollout_steps": 5000,
                   "heldout_robots": args.held_pools * args.pool,
                   "train_rollouts": int(len(Xtr)), "heldout_candidates": int(n_cand), "epochs": args.epochs,
                   "mlp": [int(Xtr.shape[1]), args.width, args.width, args.width, int(Dtr.shape[1])],
                   "mlp_params": sur.n_params, "lr": args.lr, "lr_final": args.lr_final if args.lr_final >= 0 else args.lr},
        "surrogate_evals_per_s": sur_rate, "sim_evals_per_s": sim_rate,
        "surrogate_evals_per_s_with_morphology": sur_rate_morph,
        "morphology_features_per_robot_s": t_morph / len(held_bodies),
        "screening_pass_seconds": t_screen,
        "rms_rel_error": err, "p95_rel_error": float(np.percentile(per, 95)),
        "rms_rel_error_constant_predictor": err_mean, "simulator_noise_floor": noise_floor,
        "simulator_noise_floor_x": noise_floor_x,
        "train_loss": sur.train_loss,
        "train_seconds": sur.train_seconds, "flagged": int(flagged.sum()), "simulated_after_screen": int(len(chosen)),
        "top5pct_overlap": len(true_top & pred_top) / k, "top5pct_overlap_random": k / n_cand,
        "best_true_x_in_screened": float(Dte[chosen, 0].max()), "best_true_x_overall": float(Dte[:, 0].max()),
        # the screened quantity alone: forward (x) displacement
        "x_rms_rel_error": float(np.sqrt(((pred[:, 0] - Dte[:, 0]) ** 2).mean() / (Dte[:, 0] ** 2).mean())),
        "x_rms_rel_error_constant_predictor": float(np.sqrt(((Dtr[:, 0].mean() - Dte[:, 0]) ** 2).mean() /
                                                            (Dte[:, 0] ** 2).mean())),
        "x_spearman": float(np.corrcoef(np.argsort(np.argsort(pred[:, 0])), np.argsort(np.argsort(Dte[:, 0])))[0, 1]),
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--batch", type=int, default=0, help="entries loaded ahead per lane (2, 4 or 8; 0 = default)")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per mass (1, 2 or 4; 0 = default)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--fast-diff", action="store_true", help="skip the exact coordinate difference")
    ap.add_argument("--no-table", action="store_true", help="explicit per-entry (k, L0) instead of the table")
    ap.add_argument("--split", action="store_true", help="split step form (spring pass + gather pass)")
    ap.add_argument("--wide-entries", action="store_true", help="32-bit compact entries even where 16-bit ones fit")
    ap.add_argument("--no-grid", action="store_true", help="never the structured-box step form")
    ap.add_argument("--integrator", choices=("euler", "verlet"), default="euler",
                    help="symplectic Euler (default) or Verlet, eqs. (5)-(6)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="processes of the all-cores oracle baseline (0: the available cores, at most 16; 1: skip)")
    ap.add_argument("--nx", type=int, default=400)
    ap.add_argument("--workload", choices=("cantilever", "population", "quadruped", "cube", "candidate", "surrogate",
                                           "adjoint", "frequency", "modes", "mlp"), default="cantilever")
    ap.add_argument("--mlp-rows", type=int, default=196_608, help="mlp: training rows")
    ap.add_argument("--sweep", type=lambda t: [tuple(int(v) for v in b.split("x")) for b in t.split(",")],
                    default=[(200, 40, 40), (300, 40, 40), (400, 40, 40), (400, 40, 30), (400, 40, 20), (400, 20, 40)],
                    help="frequency, modes: beams as NXxNYxNZ node counts, comma separated")
    ap.add_argument("--modes-iter", type=int, default=1_000_000, help="modes: Lanczos step cap per beam")
    ap.add_argument("--points", type=int, default=200_000, help="candidate: points of the best-candidate bar")
    ap.add_argument("--resident", action="store_true", help="one-workgroup multi-step form (systems of <= 1024 masses)")
    ap.add_argument("--adjoint-steps", type=int, default=2000, help="adjoint: rollout length")
    ap.add_argument("--pool", type=int, default=1024, help="surrogate: robots per morphology pool")
    ap.add_argument("--pools", type=int, default=8, help="surrogate: training pools (disjoint robots)")
    ap.add_argument("--held-pools", type=int, default=1, help="surrogate: held-out pools")
    ap.add_argument("--draws", type=int, default=8, help="surrogate: actuation draws simulated per robot")
    ap.add_argument("--epochs", type=int, default=150, help="surrogate: training epochs")
    ap.add_argument("--width", type=int, default=768, help="surrogate: hidden layer width")
    ap.add_argument("--lr", type=float, default=2e-3, help="surrogate: initial learning rate")
    ap.add_argument("--lr-final", type=float, default=0.0, help="surrogate: final learning rate of the cosine schedule (-1: constant)")
    ap.add_argument("--dump", default="", help="surrogate: directory to save the data set to (npz)")
    ap.add_argument("--robots", type=int, default=1024)
    ap.add_argument("--tune", action="store_true", help="run the autotuner before timing")
    ap.add_argument("--settle-ms", type=float, default=100.0,
                    help="milliseconds of the same steps on a second copy of the workload before the warm-up, "
                         "so that the timed steps run at the device's sustained clocks (0: none)")
    ap.add_argument("--calibrate-copy", type=int, default=2048, metavar="MIB",
                    help="before the timed steps, time the library's streaming copy and read kernels over "
                         "MIB MiB (the attainable-bandwidth reference and the reference kernel for the HBM "
                         "byte counters); 0 skips")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for {args.gpus}); the step of one body would shard "
              "into Morton slabs with a halo exchange, which is not implemented.", file=sys.stderr)
        sys.exit(2)

    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import torch

    if args.workload == "surrogate":
        print(json.dumps(surrogate_bench(args)), flush=True)
        return
    if args.workload == "adjoint":
        print(json.dumps(adjoint_bench(args)), flush=True)
        return
    if args.workload == "mlp":
        print(json.dumps(mlp_bench(args)), flush=True)
        return
    if args.workload == "frequency":
        print(json.dumps(frequency_bench(args)), flush=True)
        return
    if args.workload == "modes":
        print(json.dumps(modes_bench(args)), flush=True)
        return

    import workloads as W
    from paper_2207_09334_amd import cronos as CR
    from paper_2207_09334_amd import problem as PR

    stream = torch.cuda.Stream()
    flags = ((CR.NO_GRAPH if args.no_graph else 0) | (CR.FAST_DIFF if args.fast_diff else 0) |
             (CR.NO_TABLE if args.no_table else 0) | (CR.SPLIT if args.split else 0) |
             (CR.WIDE_ENTRIES if args.wide_entries else 0) | (CR.NO_GRID if args.no_grid else 0) |
             (CR.VERLET if args.integrator == "verlet" else 0) | (CR.RESIDENT if args.resident else 0))
    if args.workload == "candidate":
        w = W.candidate_bar(args.points)

        def make():
            return PR.create_points(w, stream=stream.cuda_stream, flags=flags, block_masses=args.block)[0]
        n_bodies, batched, actuated, lat = 1, False, False, None
    else:
        if args.workload == "population":
            w = W.population(args.robots)
        elif args.workload == "quadruped":
            w = W.quadruped()
        elif args.workload == "cube":
            w = W.cube_drop()
        else:
            w = W.cantilever(args.nx, 40, 40)
        lat = PR.build_lattice(w)

        def make():
            return PR.create(w, lat=lat, stream=stream.cuda_stream, flags=flags, block_masses=args.block,
                             batch=args.batch, lanes_per_mass=args.lanes, tune_steps=20 if args.tune else 0)[0]
        n_bodies, batched, actuated = len(w.bodies), len(w.bodies) > 1, w.n_groups > 0
    sim = make()
    info = CR.cronos_info(sim)
    launch = CR.cronos_launch_config(sim)
    mode = CR.cronos_launch_mode(sim)
    N, S = info["n_masses"], info["n_springs"]

    copy_gbs = read_gbs = None
    if args.calibrate_copy:
        # the library's plain streaming kernels over a buffer of known size: the bandwidth a
        # hand-written HIP copy (read + write) and read pass reach on this device (best of 5)
        copy_gbs, read_gbs = CR.cronos_stream_bandwidth(args.calibrate_copy << 20, reps=5)
    # The device raises its clocks over milliseconds of sustained work and lowers them within
    # milliseconds of idling, so a few steps timed right after a short warm-up from an idle
    # device run slower than the same steps do in a long run.  A second copy of the workload
    # measures that first (the same W warm-up and K timed steps, from idle: cold_ms_per_step),
    # then runs its steps for --settle-ms; the timed simulation's W warm-up steps follow on the
    # same stream with no idle gap, then the synchronised K timed steps.
    settle = None
    twin = None
    if args.settle_ms > 0:
        twin = make()
        torch.cuda.synchronize()
        CR.cronos_step(twin, args.warmup)
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        CR.cronos_step(twin, args.steps)
        c1.record(stream)
        c1.synchronize()
        cold_ms = c0.elapsed_time(c1)
        probe = 16
        c0.record(stream)
        CR.cronos_step(twin, probe)
        c1.record(stream)
        c1.synchronize()
        n_settle = max(1, int(math.ceil(args.settle_ms / max(c0.elapsed_time(c1) / probe, 1e-3))))
        CR.cronos_step(twin, n_settle)
        settle = {"steps": probe + n_settle, "ms": args.settle_ms, "on": "a second copy of the workload",
                  "cold_ms_per_step": cold_ms / args.steps}
    CR.cronos_step(sim, args.warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    CR.cronos_step(sim, args.steps)
    end.record(stream)
    end.synchronize()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    if twin is not None:
        twin.close()
    x, v, step = CR.cronos_read_state(sim)
    import numpy as np
    if not np.isfinite(x).all():
        print("bench.py: non-finite state after the timed steps", file=sys.stderr)
        sys.exit(1)

    sec_per_step = ms / 1e3 / args.steps
    value = S / sec_per_step
    b_kernel = kernel_bytes(N, S, launch["step_form"], actuated=actuated)
    b_formula = formula_bytes(N, S, actuated=actuated, batched=batched)
    achieved = b_kernel / sec_per_step / 1e9
    prof = profile_record(w.name, launch)
    traffic = float(prof["hbm_bytes_per_launch"]) if prof else None
    out = {
        "metric": METRIC, "value": value, "unit": "spring-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "n_bodies": n_bodies, "n_masses": N, "n_springs": S, "dt": w.dt,
                   "block_masses": launch["block_masses"], "batch": launch["batch"],
                   "persistent_groups": launch["persistent_groups"], "hip_graph": mode["hip_graph"],
                   "plain_step_us_at_creation": mode["plain_step_us"], "staged_io": mode["staged_io"],
                   "exact_difference": not args.fast_diff, "step_form": launch["step_form"],
                   "lanes_per_mass": launch["lanes_per_mass"],
                   "integrator": args.integrator},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": b_kernel,
                     "traffic_frac": None if traffic is None else traffic / sec_per_step / 1e9 / HBM_PEAK_GBS,
                     "formula_bytes_per_launch": b_formula,
                     "formula_frac": b_formula / sec_per_step / 1e9 / HBM_PEAK_GBS},
    }
    # the arithmetic ceiling: the method's issue cycles per step against one wave64 VALU
    # instruction per CU per cycle; the roofline reported is the one the step is closer to
    cyc = alu_cycles(S, actuated)
    alu = {"bound": "alu", "achieved": cyc / sec_per_step, "peak": VALU_PEAK, "unit": "wave64 VALU issue cycles/s",
           "frac": cyc / sec_per_step / VALU_PEAK, "traffic": traffic, "algorithmic_cycles_per_launch": cyc}
    if alu["frac"] > out["roofline"]["frac"]:
        hbm = out["roofline"]
        out["roofline"] = alu
        out["roofline"]["hbm"] = hbm
    else:
        out["roofline"]["alu"] = alu
    if copy_gbs is not None:
        hb = out["roofline"] if out["roofline"]["bound"] == "hbm" else out["roofline"]["hbm"]
        hb["copy_kernel_gbs"] = copy_gbs
        hb["read_kernel_gbs"] = read_gbs
        hb["frac_of_copy"] = achieved / copy_gbs
        if traffic is not None:
            hb["traffic_frac_of_copy"] = traffic / sec_per_step / 1e9 / copy_gbs
    if prof and prof.get("valu_wave_instr_per_launch"):
        # the step's other ceiling: VALU issue, one wave64 instruction per cycle per CU
        # (non-packed FP32), from the committed SQ_INSTS_VALU count of this configuration
        rate = prof["valu_wave_instr_per_launch"] / sec_per_step
        out["valu_issue"] = {"achieved": rate, "peak": VALU_PEAK, "unit": "wave64 VALU instr/s",
                             "frac": rate / VALU_PEAK, "instr_per_launch": prof["valu_wave_instr_per_launch"]}
    if settle is not None:
        out["clock_settle"] = settle
    if batched:
        out["rollouts_per_s"] = len(w.bodies) / (w.steps * sec_per_step)
        out["rollout_steps"] = w.steps
    sim.close()
    if not args.no_cpu_baseline and lat is not None:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
        if args.cpu_procs != 1 and len(w.bodies) == 1:
            procs = args.cpu_procs or min(16, len(os.sched_getaffinity(0)))
            out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(w, max(1, args.cpu_steps // 2), procs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
