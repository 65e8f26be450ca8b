"""Throughput of the cascaded D2Q9 LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Headline (`value`): MLUPS of the plain FP32 step on the lid-driven cavity
4096 x 4096 (Re 1000, lid 0.1, tau 1.7288; seeded density noise 1e-6), with
the lattices resident in HBM: W untimed steps, then exactly K steps (default
100 000, the study's step count at its largest grid) timed with HIP events on
the library's stream (lbm_step fuses four steps per launch in FP64 and FP32,
two in FP16/BF16).  One JSON line on stdout, also carrying:

  roofline      the dominant kernel, the four-step FP32 launch.  It keeps
                the intermediate steps on chip and moves 18 B per update, so
                it is bound by VALU issue, not by HBM: bound "alu", achieved =
                the method's own operations per launch (94 VALU operations
                per FP32 cell update at the default rates, times the four
                updates of every node) over the launch's average duration
                (HIP events between the whole groups and any remainder of K),
                against 39.32 T VALU operations/s (256 CUs x 4 SIMDs x 16
                lanes x 2.4 GHz; packed FP32 is not used).  Beside it: the
                VALU issue fraction from the committed SQ_INSTS_VALU count,
                flops against the FP32 vector peaks, and the HBM side: the
                single-pass algorithmic rate at 72 B per update as a ratio of
                8 TB/s (alg_hbm_ratio, above 1 by construction), the bytes the
                launch actually moves and their fraction of 8 TB/s and of the
                copy bandwidth measured in the same run;
  copy          a plain device-to-device copy of 2 x 2 GiB timed in the run;
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the headline cavity;
  cpu_plan      the oracle on the other configurations (all host threads and
                one), the host's copy bandwidth, the CPU model, and the GPU /
                oracle ratio per configuration;
  sizes         the same cavity at 1024^2 and 2048^2 (Re 1000) and 4096^2
                (Re 5000), FP32, each timed for at least 0.5 s right before
                the headline (so that the headline is timed in the GPU's
                settled clock state), with the FP32 velocity and strain-rate
                error against the FP64 path;
  flows         FP32 Taylor-Green 8192^2 and Poiseuille channels (the
                256 x 64 configuration and a 8192 x 2048 channel);
  forms         FP16/BF16 deviation storage (nearest and stochastic
                rounding) on Taylor-Green 8192^2 (MLUPS, roofline) with the
                errors against the FP64 path on Taylor-Green 512^2 after 20k
                steps at tau 0.8 and 0.55; the forward + adjoint rollout on
                512 x 512 (T = 2000, checkpoint every 100; and with every
                state kept, so that the backward recomputes nothing) and
                2048 x 2048 (T = 400) with the FP32 gradient's error against
                the FP64 gradient; the adjoint pair launch at 2048^2 on its
                own, with its HBM roofline (168 B per node and launch); the
                single-step launch in FP32, FP16 and BF16.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# Algorithmic bytes per cell update: nine populations read, nine written.
BYTES_PER_UPDATE = {"fp64": 144, "fp32": 72, "fp16": 36, "bf16": 36}
METRIC = "MLUPS + % HBM peak, FP32 vs FP16-storage; fwd+adjoint MLUPS at fixed error"
STEP_SOURCES = ["paper_1202_6351_amd/csrc/lbm_kernels.hip", "paper_1202_6351_amd/csrc/cascade.h",
                "paper_1202_6351_amd/csrc/lbm_launch.h", "paper_1202_6351_amd/csrc/lbm_api.hip"]
PROFILES = os.path.join(ROOT, "profiles")
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (non-packed lane
# operations per second; one wave64 instruction per SIMD every 4 cycles).
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
FP32_PEAK_TFLOPS_NONPACKED = 2 * VALU_PEAK_OPS / 1e12  # every lane an FMA: 78.6
FP32_PEAK_TFLOPS_PUBLISHED = 157.3  # packed FP32 FMA
# One FP32 cell update of the kernels' factorised collision, without body
# force and at omega_3 = omega_6 = omega_7 = omega_8 = 1 (their multiplies
# left out): 94 VALU operations (30 add, 16 sub, 8 mul, 39 fma, 1 rcp), 133
# flops with an fma counted as two.  The 16-bit forms add the conversions:
# bfloat16 one per population loaded (a shift) and one per population stored
# (112); binary16 one per population loaded, while eight of the nine stores
# fold their conversion into the final fma (v_fma_mixlo_f16), so 104.
COLLISION_OPS = {"fp32": 94, "fp64": 94, "fp16": 104, "bf16": 112}
COLLISION_FLOPS_FP32 = 133


def updates_per_launch(storage: str) -> int:
    """Steps the library fuses per launch: four in FP64 and FP32, two in
    16-bit storage."""
    return 2 if storage in ("fp16", "bf16") else 4


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in STEP_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_value(name, key):
    """A per-launch figure from a committed counter summary under profiles/,
    if the counters were taken on the current kernel sources (else None)."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel_source_sha256:\s*(\w+)", txt)
    m_val = re.search(key + r":\s*([0-9.eE+]+)", txt)
    if not (m_hash and m_val) or m_hash.group(1) != kernel_hash():
        return None
    return float(m_val.group(1))


def timed_steps(lat, steps, warmup, group):
    """Time exactly `steps` steps with HIP events on the library's stream.
    Returns (seconds for all steps, seconds for the whole groups, number of
    group launches): the remainder of steps modulo the group runs after an
    intermediate event, so the second figure covers one kernel only."""
    import torch
    lat.step(warmup)
    torch.cuda.synchronize()
    s = lat.stream
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    whole = steps - steps % group
    e0.record(s)
    lat.step(whole)
    e1.record(s)
    lat.step(steps - whole)
    e2.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e2) / 1e3, e0.elapsed_time(e1) / 1e3, whole // group


def timed_for(lat, group, min_seconds=0.5):
    """(MLUPS, seconds per launch) of whole-group launches, timed with HIP
    events over at least min_seconds after a short calibration."""
    nodes = lat.params.nx * lat.params.ny
    _, dt, n = timed_steps(lat, 8 * group, 2 * group, group)
    launches = max(8, int(math.ceil(min_seconds / max(dt / n, 1e-7))))
    _, dt, n = timed_steps(lat, launches * group, 0, group)
    return nodes * group * n / dt / 1e6, dt / n


def cavity_lattice(n, storage, re=1000.0):
    import workloads as W
    from paper_1202_6351_amd import Lattice, Params
    tau = W.cavity_tau(n, 0.1, re)
    p = Params(n, n, tau=tau, bc=("wall",) * 4, wall_u=(0, 0, 0, 0.1), storage=storage)
    lat = Lattice(p, device="cuda:0")
    lat.init_equilibrium(*W.at_rest(n, n, density_noise=1e-6, seed=2))
    return lat, tau


def taylor_green_lattice(n, storage, u0=0.05, tau=0.8, rounding="nearest"):
    import workloads as W
    from paper_1202_6351_amd import Lattice, Params
    lat = Lattice(Params(n, n, tau=tau, storage=storage, rounding=rounding, seed=1), device="cuda:0")
    lat.init_equilibrium(*W.taylor_green(n, u0, noise=1e-5, seed=0))
    return lat


def poiseuille_lattice(nx, ny, storage, tau=0.8):
    import workloads as W
    from paper_1202_6351_amd import Lattice, Params
    F = W.poiseuille_force(tau, 0.05, ny)
    lat = Lattice(Params(nx, ny, tau=tau, fx=F, bc=("periodic", "periodic", "wall", "wall"), storage=storage),
                  device="cuda:0")
    lat.init_equilibrium(*W.at_rest(nx, ny))
    return lat


def field_errors(m, ref):
    """Velocity (Sec. III norm) and strain-rate relative errors of m against
    ref (numpy node fields)."""
    import numpy as np
    den_u = np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2).sum()
    eu = np.sqrt((m["ux"] - ref["ux"]) ** 2 + (m["uy"] - ref["uy"]) ** 2).sum() / den_u
    s_num = sum(np.abs(m[k] - ref[k]).sum() for k in ("sxx", "syy", "sxy"))
    s_den = sum(np.abs(ref[k]).sum() for k in ("sxx", "syy", "sxy"))
    return float(f"{eu:.3e}"), float(f"{s_num / s_den:.3e}")


def copy_bandwidth(nbytes=2 << 30, reps=10):
    """Device-to-device copy of nbytes (read nbytes, write nbytes), timed with
    HIP events: GB/s of bytes moved."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1e3
    del a, b
    torch.cuda.empty_cache()
    return round(2 * nbytes * reps / dt / 1e9, 1)


def alu_block(storage, nodes, per_launch):
    """VALU roofline of a step launch from the method's operation count."""
    grp = updates_per_launch(storage)
    ops = COLLISION_OPS[storage]
    achieved = ops * grp * nodes / per_launch / 1e12
    return {"bound": "alu", "achieved": round(achieved, 2), "peak": round(VALU_PEAK_OPS / 1e12, 2),
            "unit": "TOP/s", "frac": round(achieved * 1e12 / VALU_PEAK_OPS, 4), "ops_per_update": ops}


def cpu_baseline(n, tau, budget_s=10.0):
    """The FP64 oracle on the headline cavity, first steps from the same
    initial state, on all host threads, for about budget_s of stepping (after
    one untimed step that starts the thread pool)."""
    import oracle
    import workloads as W
    p = oracle.Params(n, n, tau=tau, bc=(1, 1, 1, 1), wall_u=(0, 0, 0, 0.1))
    f = oracle.init_state(p, *W.at_rest(n, n, density_noise=1e-6, seed=2))
    f = oracle.step(p, f, 1)
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        f = oracle.step(p, f, 4)
        steps += 4
    dt = time.perf_counter() - t0
    return {"value": round(n * n * steps / dt / 1e6, 2), "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"FP64 oracle, lid-driven cavity {n}x{n} Re 1000, {steps} steps after the first "
                      f"from the benchmark's initial state ({dt:.1f} s)"}


# The oracle's share of the plan: (name, builder, steps on all threads, steps
# on one thread).  Builders return (oracle params, initial state).
def _plan_cases():
    import oracle
    import workloads as W

    def tg64():
        p = oracle.Params(64, 64, tau=0.8)
        return p, oracle.init_state(p, *W.taylor_green(64, 0.01, noise=1e-5, seed=0))

    def pois():
        p = oracle.Params(256, 64, tau=0.8, fx=W.poiseuille_force(0.8, 0.05, 64), bc=(0, 0, 1, 1))
        return p, oracle.init_state(p, *W.at_rest(256, 64))

    def cav1024():
        p = oracle.Params(1024, 1024, tau=W.cavity_tau(1024, 0.1, 1000.0), bc=(1, 1, 1, 1), wall_u=(0, 0, 0, 0.1))
        return p, oracle.init_state(p, *W.at_rest(1024, 1024, density_noise=1e-6, seed=2))

    def tg512():
        p = oracle.Params(512, 512, tau=0.8)
        return p, oracle.init_state(p, *W.taylor_green(512, 0.05, noise=1e-5, seed=0))

    return [("taylor_green_64x64_fp64", tg64, 1000, 1000),
            ("poiseuille_256x64_tau0.8", pois, 8000, 2000),
            ("cavity_1024x1024_re1000", cav1024, 200, 12),
            ("taylor_green_512x512", tg512, 200, 40)]


def _oracle_plan_worker(single: bool):
    """Runs in a child process (its own OpenMP thread count): oracle MLUPS
    per plan configuration."""
    import oracle
    out = {}
    for name, build, steps, steps1 in _plan_cases():
        p, f = build()
        n = steps1 if single else steps
        f = oracle.step(p, f, 1)
        t0 = time.perf_counter()
        oracle.step(p, f, n)
        dt = time.perf_counter() - t0
        out[name] = {"steps": n, "seconds": round(dt, 3), "mlups": round(p.nx * p.ny * n / dt / 1e6, 2)}
    out["threads"] = oracle.num_threads()
    print(json.dumps(out))


def host_copy_bandwidth(nbytes=1 << 30, reps=5):
    """Host memory copy bandwidth with torch's CPU threads (GB/s moved)."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64)
    b = torch.empty_like(a)
    b.copy_(a)
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    dt = time.perf_counter() - t0
    return round(2 * nbytes * reps / dt / 1e9, 1), torch.get_num_threads()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def gpu_plan_rates():
    """GPU MLUPS on the plan's configurations, FP64 (the oracle's arithmetic)
    and the configuration's own storage, each timed for at least 0.5 s."""
    import torch
    out = {}
    for name, mk, storages in (
            ("taylor_green_64x64_fp64", lambda s: taylor_green_lattice(64, s, u0=0.01), ("fp64",)),
            ("poiseuille_256x64_tau0.8", lambda s: poiseuille_lattice(256, 64, s), ("fp64", "fp32")),
            ("cavity_1024x1024_re1000", lambda s: cavity_lattice(1024, s)[0], ("fp64", "fp32")),
            ("taylor_green_512x512", lambda s: taylor_green_lattice(512, s), ("fp64", "fp32", "fp16", "bf16"))):
        out[name] = {}
        for st in storages:
            lat = mk(st)
            out[name][st] = round(timed_for(lat, updates_per_launch(st))[0], 1)
            del lat
        torch.cuda.empty_cache()
    return out


def cpu_plan(gpu_rates):
    """The oracle on the plan's configurations, on all host threads and on one,
    in child processes; host copy bandwidth; GPU / oracle ratios."""
    res = {}
    for single in (False, True):
        env = dict(os.environ)
        if single:
            env["OMP_NUM_THREADS"] = "1"
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-plan-worker",
                            "single" if single else "all"], capture_output=True, text=True, env=env,
                           timeout=300)
        if r.returncode != 0:
            raise RuntimeError(f"oracle plan worker failed: {r.stderr[-2000:]}")
        res["one" if single else "all"] = json.loads(r.stdout.strip().splitlines()[-1])
    bw, bw_threads = host_copy_bandwidth()
    table = {}
    for name in res["all"]:
        if name == "threads":
            continue
        a, o = res["all"][name], res["one"][name]
        g = gpu_rates.get(name, {})
        table[name] = {"oracle_mlups": a["mlups"], "oracle_steps": a["steps"], "oracle_seconds": a["seconds"],
                       "oracle_mlups_1core": o["mlups"],
                       "oracle_frac_of_host_copy": round(a["mlups"] * 144 / 1e3 / bw, 4),
                       "gpu_mlups": g,
                       "gpu_fp64_over_oracle": (round(g["fp64"] / a["mlups"], 1) if "fp64" in g else None)}
    return {"kind": "oracle", "threads": res["all"]["threads"], "cpu_model": cpu_model(),
            "host_copy_gbs": bw, "host_copy_threads": bw_threads,
            "oracle_bytes_per_update": 144, "configs": table}


def precision_errors(n=512, steps=20000, tau=0.8):
    """Velocity and strain-rate relative error of FP32, FP16 and BF16 storage
    against the FP64 path, Taylor-Green n x n, U0 0.05, noise 1e-5."""
    import torch
    out = {}
    ref = taylor_green_lattice(n, "fp64", tau=tau).step(steps).macroscopic()
    ref = {k: v.cpu().numpy() for k, v in ref.items()}
    for storage, rounding in (("fp32", "nearest"), ("fp16", "nearest"), ("bf16", "nearest"),
                              ("fp16", "stochastic"), ("bf16", "stochastic")):
        m = taylor_green_lattice(n, storage, tau=tau, rounding=rounding).step(steps).macroscopic()
        m = {k: v.cpu().numpy() for k, v in m.items()}
        eu, es = field_errors(m, ref)
        key = storage if rounding == "nearest" else f"{storage}_sr"
        out[key] = {"u_rel_err": eu, "strain_rel_err": es}
    torch.cuda.synchronize()
    return {"workload": f"taylor_green_{n}x{n}_u0.05_tau{tau}_{steps}steps", "reference": "fp64 GPU path",
            **out}


def adjoint_rollout(n=512, T=2000, every=100):
    """Forward + adjoint of the differentiable rollout (n x n periodic, force
    field N(0, 1e-6^2) seed 4, u0 = 0, Taylor-Green target U0 = 0.02), FP32
    timed (second pass), with the FP32 gradient against the FP64 one."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1202_6351_amd import Params, rollout
    k = 2 * math.pi / n
    nu = (0.8 - 0.5) / 3
    x = np.arange(n)[None, :]
    y = np.arange(n)[:, None]
    dec = math.exp(-2 * nu * k * k * T)
    tgt = torch.from_numpy(np.stack([-0.02 * np.cos(k * x) * np.sin(k * y) * dec,
                                     0.02 * np.sin(k * x) * np.cos(k * y) * dec])).cuda()
    res = {}
    for storage in ("fp32", "fp64"):
        real = torch.float32 if storage == "fp32" else torch.float64
        p = Params(n, n, tau=0.8, storage=storage)
        # the first pass pays the device allocations of snapshots and the
        # segment buffer; the second one (same sizes, cached) is timed
        for _ in range(2 if storage == "fp32" else 1):
            F = torch.from_numpy(W.force_field(n, n, 1e-6, seed=4)).to("cuda", real).requires_grad_(True)
            u0 = torch.zeros(2, n, n, dtype=real, device="cuda", requires_grad=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, u = rollout(p, F, u0, T, checkpoint_every=every)
            loss = ((u - tgt) ** 2).sum(dim=0).mean()
            loss.backward()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        res[storage] = (dt, F.grad.double().cpu().numpy(), u0.grad.double().cpu().numpy())
        del F, u0, u, loss
        torch.cuda.empty_cache()
    dt = res["fp32"][0]
    errF = np.abs(res["fp32"][1] - res["fp64"][1]).sum() / np.abs(res["fp64"][1]).sum()
    erru = np.abs(res["fp32"][2] - res["fp64"][2]).sum() / np.abs(res["fp64"][2]).sum()
    return {"workload": f"rollout_{n}x{n}_fp32_T{T}_ckpt{every}", "mlups": round(n * n * T / dt / 1e6, 1),
            "seconds": round(dt, 3), "grad_force_rel_err_vs_fp64": float(f"{errF:.3e}"),
            "grad_u0_rel_err_vs_fp64": float(f"{erru:.3e}")}


# Adjoint launches timed on their own: steps per launch -> (kernel,
# algorithmic bytes per node and launch, counter summaries under profiles/).
# Pair: two states 72, cotangent in 36 and out 36, force 8, force gradient
# read and written 16.  Quad: four states 144 and the same 96 besides.
ADJOINT_LAUNCHES = {
    2: ("k_adjoint_step2<float> (two adjoint steps per launch)", 168,
        "traffic_adjoint2_fp32_2048.txt", "valu_adjoint2_fp32_2048.txt"),
    4: ("k_adjoint_step4<float> (four adjoint steps per launch)", 240,
        "traffic_adjoint4_fp32_2048.txt", "valu_adjoint4_fp32_2048.txt"),
}


def adjoint_launch_roofline(n=2048, steps=2, launches=50, copy_gbs=None):
    """One adjoint launch of `steps` steps (the pair k_adjoint_step2 or, on
    lattices of 200 000 nodes and more, the four-step k_adjoint_step4) on an
    n x n periodic FP32 lattice with a force field, timed with HIP events over
    `launches` launches: its HBM roofline at the algorithmic bytes per node
    and launch."""
    import torch
    import workloads as W
    from paper_1202_6351_amd import Lattice, Params
    kernel, bpn, f_traffic, f_valu = ADJOINT_LAUNCHES[steps]
    lat = Lattice(Params(n, n, tau=0.8, storage="fp32"), device="cuda:0",
                  force=torch.from_numpy(W.force_field(n, n, 1e-6, seed=4)))
    lat.init_equilibrium(*W.taylor_green(n, 0.02))
    states = [lat.new_lattice() for _ in range(steps + 1)]
    lat.step_sequence(lat.snapshot(), states)
    mu_a, mu_b = lat.new_cotangent(), lat.new_cotangent()
    mu_a.normal_()
    gF = torch.zeros((2, n, n), dtype=torch.float32, device="cuda")
    seq = states[:steps]
    lat.adjoint_sequence(seq, mu_a, mu_b, gF)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    for _ in range(launches):
        lat.adjoint_sequence(seq, mu_a, mu_b, gF)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    per = e0.elapsed_time(e1) / 1e3 / launches
    alg = bpn * n * n / per / 1e9
    traffic = counter_value(f_traffic, "traffic_bytes_per_launch") if n == 2048 else None
    valu = counter_value(f_valu, "valu_wave_instructions_per_launch") if n == 2048 else None
    out = {"kernel": kernel, "workload": f"adjoint_{n}x{n}_fp32",
           "launch_us": round(per * 1e6, 2), "adjoint_glups": round(steps * n * n / per / 1e9, 2),
           "roofline": {"bound": "hbm", "achieved": round(alg, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(alg / HBM_PEAK_GBS, 4), "traffic": None if traffic is None else round(traffic),
                        "alg_bytes_per_node": bpn,
                        "vs_copy": None if not copy_gbs else round(alg / copy_gbs, 4)}}
    if valu is not None:
        out["valu_issue"] = {"lane_instructions_per_node_step": round(valu * 64 / (steps * n * n), 1),
                             "frac": round(valu * 64 / per / VALU_PEAK_OPS, 4)}
    return out


def single_step_rates(n=8192, copy_gbs=None, min_seconds=0.5):
    """One step per launch (lbm_step_between, the single-step kernel) on the
    Taylor-Green n^2 lattice in FP32, FP16 and BF16: the launch reads and
    writes the state once, so HBM bounds it and the 16-bit storage halves
    its bytes."""
    import torch
    out = {}
    for storage in ("fp32", "fp16", "bf16"):
        lat = taylor_green_lattice(n, storage)
        a, b = lat.lat[0], lat.lat[1]
        if lat.current is not a:
            a, b = b, a
        s = lat.stream
        for _ in range(4):
            lat.step_between(a, b)
            lat.step_between(b, a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(4):
            lat.step_between(a, b)
            lat.step_between(b, a)
        e1.record(s)
        torch.cuda.synchronize()
        pairs = max(4, int(math.ceil(min_seconds / max(e0.elapsed_time(e1) / 1e3 / 4, 1e-7))))
        e0.record(s)
        for _ in range(pairs):
            lat.step_between(a, b)
            lat.step_between(b, a)
        e1.record(s)
        torch.cuda.synchronize()
        dt = e0.elapsed_time(e1) / 1e3 / (2 * pairs)
        moved = BYTES_PER_UPDATE[storage] * n * n / dt / 1e9
        out[storage] = {"mlups": round(n * n / dt / 1e6, 1), "launch_us": round(dt * 1e6, 2),
                        "moved_gbs": round(moved, 1), "moved_frac": round(moved / HBM_PEAK_GBS, 4)}
        if copy_gbs:
            out[storage]["moved_vs_copy"] = round(moved / copy_gbs, 4)
        del lat, a, b
        torch.cuda.empty_cache()
    out["workload"] = f"taylor_green_{n}x{n}, one step per launch (lbm_step_between)"
    return out


def copy_calibration(nbytes=1 << 30):
    """A plain elementwise copy kernel of known size (reads and writes nbytes),
    so that counter runs can scale the step kernel's FETCH_SIZE / WRITE_SIZE
    by what the same counters read for it."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()


def cavity_errors(n, re, steps):
    """FP32 against the FP64 path on the cavity after `steps` steps (the
    FP64 path equals the oracle to 1e-12 in the parity tests)."""
    m32 = {k: v.cpu().numpy() for k, v in cavity_lattice(n, "fp32", re)[0].step(steps).macroscopic().items()}
    m64 = {k: v.cpu().numpy() for k, v in cavity_lattice(n, "fp64", re)[0].step(steps).macroscopic().items()}
    eu, es = field_errors(m32, m64)
    return {"steps": steps, "u_rel_err": eu, "strain_rel_err": es, "reference": "fp64 GPU path"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--n", type=int, default=4096, help="cavity size of the headline run")
    ap.add_argument("--only", choices=["fp32", "fp16", "bf16", "fp64", "rollout", "rollout_keep_all", "rollout2048", "adjoint2048",
                                       "single"],
                    default=None, help="time one storage mode, the forward + adjoint rollout, the adjoint launches or the single-step "
                    "launches, only (profiling runs)")
    ap.add_argument("--rounding", choices=["nearest", "stochastic"], default="nearest",
                    help="16-bit rounding of an --only fp16/bf16 run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--oracle-plan-worker", choices=["all", "single"], default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_plan_worker:
        _oracle_plan_worker(args.oracle_plan_worker == "single")
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU domain decomposition is a design note only).", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        copy_calibration()
    if args.only == "rollout":
        print(json.dumps({"only": "rollout", **adjoint_rollout()}))
        return
    if args.only == "rollout_keep_all":
        print(json.dumps({"only": "rollout_keep_all", **adjoint_rollout(512, 2000, 2000)}))
        return
    if args.only == "rollout2048":
        print(json.dumps({"only": "rollout2048", **adjoint_rollout(2048, 400, 100)}))
        return
    if args.only == "single":
        print(json.dumps({"only": "single", **single_step_rates(copy_gbs=copy_bandwidth())}))
        return
    if args.only == "adjoint2048":
        print(json.dumps({"only": "adjoint2048", "pair": adjoint_launch_roofline(2048, 2),
                          "quad": adjoint_launch_roofline(2048, 4, launches=25)}))
        return

    if args.only in ("fp16", "bf16", "fp64"):
        n = 8192 if args.only != "fp64" else 4096
        rounding = args.rounding if args.only != "fp64" else "nearest"
        lat = (taylor_green_lattice(n, args.only, rounding=rounding) if args.only != "fp64"
               else cavity_lattice(n, "fp64")[0])
        grp = updates_per_launch(args.only)
        dt, dt_main, launches = timed_steps(lat, args.steps, args.warmup, grp)
        mlups = n * n * args.steps / dt / 1e6
        gbs = BYTES_PER_UPDATE[args.only] * n * n * launches / dt_main / 1e9 if launches else None
        print(json.dumps({"only": args.only, "rounding": rounding, "n": n, "mlups": round(mlups, 1),
                          "updates_per_launch": grp, "moved_gbs": None if gbs is None else round(gbs, 1),
                          "launch_us": round(dt_main / launches * 1e6, 2) if launches else None}))
        return

    n = args.n
    grp = updates_per_launch("fp32")
    if args.steps < grp:
        raise SystemExit(f"--steps must be at least {grp} (one fused launch)")
    copy_gbs = copy_bandwidth(reps=20)
    forms_on = args.only is None and not args.no_forms
    lat, tau = cavity_lattice(n, "fp32")
    size_runs, size_lats = {}, []
    if forms_on:
        # The other grids and Reynolds number of the cavity throughput study,
        # timed first (at least 0.5 s each), with no idle gap before the
        # headline's warmup: started from idle, the GPU's clock runs through
        # a power-management transient (launches up to a third slower for
        # about 30 ms), which a short headline run would otherwise fall in.
        for ns, re in ((1024, 1000.0), (2048, 1000.0), (4096, 5000.0)):
            ls, _ = cavity_lattice(ns, "fp32", re)
            size_runs[(ns, re)] = timed_for(ls, grp)
            size_lats.append(ls)
    dt, dt_main, launches = timed_steps(lat, args.steps, args.warmup, grp)
    del size_lats
    mlups = n * n * args.steps / dt / 1e6
    per_launch = dt_main / launches
    nodes = n * n
    moved = BYTES_PER_UPDATE["fp32"] * nodes / per_launch / 1e9  # the state read and written once per launch
    alg = moved * grp  # single pass: 72 B per cell update
    d = lat.diagnostics()  # raises on a non-finite state
    headline = n == 4096
    traffic = counter_value("traffic_step4_fp32_cavity4096.txt", "traffic_bytes_per_launch") if headline else None
    valu = counter_value("valu_step4_fp32_cavity4096.txt", "valu_wave_instructions_per_launch") if headline else None
    del lat
    torch.cuda.empty_cache()
    roof = alu_block("fp32", nodes, per_launch)
    roof.update({
        "traffic": None if traffic is None else round(traffic),
        "kernel": "k_step4<float> (four steps per launch)", "launch_us": round(per_launch * 1e6, 2),
        "updates_per_launch": grp,
        "valu_issue": None if valu is None else {
            "lane_instructions_per_update": round(valu * 64 / (grp * nodes), 1),
            "achieved_tops": round(valu * 64 / per_launch / 1e12, 2),
            "frac": round(valu * 64 / per_launch / VALU_PEAK_OPS, 4)},
        "flops": {"per_update": COLLISION_FLOPS_FP32,
                  "achieved_tflops": round(COLLISION_FLOPS_FP32 * grp * nodes / per_launch / 1e12, 2),
                  "peak_tflops_nonpacked": round(FP32_PEAK_TFLOPS_NONPACKED, 1),
                  "peak_tflops_published_packed": FP32_PEAK_TFLOPS_PUBLISHED},
        "hbm": {"alg_bytes_per_update": BYTES_PER_UPDATE["fp32"], "alg_gbs": round(alg, 1),
                "alg_hbm_ratio": round(alg / HBM_PEAK_GBS, 4),
                "moved_bytes_per_update": BYTES_PER_UPDATE["fp32"] / grp, "moved_gbs": round(moved, 1),
                "moved_frac": round(moved / HBM_PEAK_GBS, 4), "copy_gbs": copy_gbs,
                "moved_vs_copy": round(moved / copy_gbs, 4)},
        "note": f"{grp} steps per launch keep the intermediate states on chip: the launch moves "
                f"{BYTES_PER_UPDATE['fp32'] / grp:g} B per update and is bound by VALU issue.  frac is the "
                "method's own operations against the VALU issue peak; valu_issue.frac counts every issued "
                "instruction (recompute rings, staging, addressing included); alg_hbm_ratio is the "
                "single-pass 72 B/update rate over 8 TB/s, which temporal blocking lets exceed 1."})
    line = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"cavity_{n}x{n}_re1000_fp32", "nx": n, "ny": n, "tau": round(tau, 6),
                   "lid_u": 0.1, "storage": "fp32", "bc": "halfway bounce-back walls, moving lid"},
        "roofline": roof,
        "copy": {"gbs": copy_gbs, "what": "device-to-device copy, 2 GiB read + 2 GiB written, HIP events"},
        "mass_drift_rel": float(f"{abs(d[0] / nodes - 1.0):.2e}"),
    }
    if forms_on:
        sizes = {}
        for (ns, re), (m, pl) in size_runs.items():
            sizes[f"cavity_{ns}x{ns}_re{int(re)}_fp32"] = {
                "mlups": round(m, 1), "launch_us": round(pl * 1e6, 2), "roofline": alu_block("fp32", ns * ns, pl),
                "error_vs_fp64": cavity_errors(ns, re, 2000)}
            torch.cuda.empty_cache()
        sizes[f"cavity_{n}x{n}_re1000_fp32"] = {"error_vs_fp64": cavity_errors(n, 1000.0, 2000)}
        line["sizes"] = sizes
        flows = {}
        for key, mk in (("taylor_green_8192x8192_fp32", lambda: taylor_green_lattice(8192, "fp32")),
                        ("poiseuille_256x64_fp32", lambda: poiseuille_lattice(256, 64, "fp32")),
                        ("poiseuille_256x64_fp64", lambda: poiseuille_lattice(256, 64, "fp64")),
                        ("poiseuille_8192x2048_fp32", lambda: poiseuille_lattice(8192, 2048, "fp32"))):
            lf = mk()
            st = lf.params.storage
            m, pl = timed_for(lf, updates_per_launch(st))
            flows[key] = {"mlups": round(m, 1), "launch_us": round(pl * 1e6, 2),
                          "roofline": alu_block(st, lf.params.nx * lf.params.ny, pl),
                          "alg_hbm_ratio": round(m * BYTES_PER_UPDATE[st] / 1e3 / HBM_PEAK_GBS, 4)}
            del lf
            torch.cuda.empty_cache()
        line["flows"] = flows
        forms = {}
        for storage in ("fp16", "bf16"):
            for rounding in ("nearest", "stochastic"):
                l16 = taylor_green_lattice(8192, storage, rounding=rounding)
                g16 = updates_per_launch(storage)
                m16, pl16 = timed_for(l16, g16)
                moved16 = BYTES_PER_UPDATE[storage] * 8192 * 8192 / pl16 / 1e9
                alg16 = BYTES_PER_UPDATE[storage] * m16 / 1e3
                key = f"{storage}_dev" if rounding == "nearest" else f"{storage}_dev_sr"
                roof16 = alu_block(storage, 8192 * 8192, pl16)
                if storage == "fp16" and rounding == "nearest":
                    v16 = counter_value("valu_step2_fp16_taylor_green8192.txt", "valu_wave_instructions_per_launch")
                    t16 = counter_value("traffic_step2_fp16_taylor_green8192.txt", "traffic_bytes_per_launch")
                    roof16["traffic"] = None if t16 is None else round(t16)
                    roof16["valu_issue"] = None if v16 is None else {
                        "lane_instructions_per_update": round(v16 * 64 / (g16 * 8192 * 8192), 1),
                        "frac": round(v16 * 64 / pl16 / VALU_PEAK_OPS, 4)}
                forms[key] = {"workload": "taylor_green_8192x8192", "rounding": rounding,
                              "mlups": round(m16, 1), "updates_per_launch": g16, "launch_us": round(pl16 * 1e6, 2),
                              "roofline": roof16,
                              "alg_gbs": round(alg16, 1), "alg_hbm_ratio": round(alg16 / HBM_PEAK_GBS, 4),
                              "moved_gbs": round(moved16, 1), "moved_frac": round(moved16 / HBM_PEAK_GBS, 4),
                              "moved_vs_copy": round(moved16 / copy_gbs, 4)}
                del l16
                torch.cuda.empty_cache()
        forms["single_step"] = single_step_rates(copy_gbs=copy_gbs)
        forms["error_vs_fp64"] = precision_errors()
        forms["error_vs_fp64_tau0.55"] = precision_errors(tau=0.55)
        forms["fwd_adjoint"] = adjoint_rollout()
        # every state kept (checkpoint interval = T: 2001 FP32 states of 512^2,
        # 18.9 GB): the backward runs the adjoint only, with no recompute
        forms["fwd_adjoint_keep_all"] = adjoint_rollout(512, 2000, 2000)
        forms["fwd_adjoint_2048"] = adjoint_rollout(2048, 400, 100)
        forms["adjoint_pair_2048"] = adjoint_launch_roofline(2048, 2, copy_gbs=copy_gbs)
        forms["adjoint_quad_2048"] = adjoint_launch_roofline(2048, 4, launches=25, copy_gbs=copy_gbs)
        line["forms"] = forms
    if args.only is None and not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(n, tau)
        line["cpu_plan"] = cpu_plan(gpu_plan_rates())
    print(json.dumps(line))


if __name__ == "__main__":
    main()
