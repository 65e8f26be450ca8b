"""Throughput of the cascaded D2Q9 LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Headline (`value`): MLUPS of the plain FP32 step on the lid-driven cavity
4096 x 4096 (Re 1000, lid 0.1, tau 1.7288; seeded density noise 1e-6), with
the lattices resident in HBM: W untimed steps, then exactly K steps (default
100 000, the study's step count at its largest grid) timed with
HIP events on the library's stream (lbm_step fuses four steps per launch in
FP64 and FP32, two in FP16/BF16).  One JSON line on stdout, also carrying:
  roofline      the dominant kernel (the four-step FP32 launch) against
                MI355X's 8 TB/s: its algorithmic bytes per launch -- the
                method's 72 B per FP32 cell update (nine populations read and
                nine written) times the four updates of every node -- over
                its measured average duration (an event between the whole
                groups and any remainder of K separates the dominant
                launches).  Fusing four steps moves only a quarter of those
                bytes (the state read and written once per launch, 18 B per
                update), so frac can exceed 1; the bytes actually moved and
                their rate are reported beside it, and so is the VALU issue
                rate from the committed SQ_INSTS_VALU count against the
                chip's 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz;
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same cavity;
  sizes         MLUPS of the same cavity at 1024^2 and 2048^2 (Re 1000) and
                at 4096^2, Re 5000 (2100 steps each);
  forms         FP16/BF16 deviation storage, round-to-nearest and
                stochastic rounding, on Taylor-Green 8192 x 8192 (MLUPS;
                algorithmic rate at 36 B per cell update and the rate of the
                bytes moved, 36 B per node per two-step launch) with their
                velocity and
                strain-rate error against the FP64 path on Taylor-Green
                512 x 512 after 20k steps at tau 0.8 and 0.55; forward + adjoint rollout MLUPS on
                512 x 512 FP32 (T = 2000, checkpoint every 100) with the FP32
                gradient's relative error against the FP64 gradient.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# Algorithmic bytes per cell update (nine populations read, nine written),
# which is also what one node moves through HBM per launch: a launch reads
# and writes the state once and advances every node by updates_per_launch
# steps (the library's grouping).
BYTES_PER_NODE = {"fp64": 144, "fp32": 72, "fp16": 36, "bf16": 36}
METRIC = "MLUPS + % HBM peak, FP32 vs FP16-storage; fwd+adjoint MLUPS at fixed error"
STEP_SOURCES = ["paper_1202_6351_amd/csrc/lbm_kernels.hip", "paper_1202_6351_amd/csrc/cascade.h",
                "paper_1202_6351_amd/csrc/lbm_launch.h", "paper_1202_6351_amd/csrc/lbm_api.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step4_fp32_cavity4096.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_step4_fp32_cavity4096.txt")
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (non-packed lane
# instructions per second).
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# One FP32 collision without body force in the kernels' factorised form, at
# the benchmark's omega_3 = omega_6 = omega_7 = omega_8 = 1 (the multiplies by
# omega_6..8 are then left out): 97 VALU operations (31 add, 17 sub, 10 mul,
# 38 fma, 1 rcp), 135 flops with an fma counted as two.  With other rates:
# 100 operations, 138 flops.
COLLISION_OPS_FP32, COLLISION_FLOPS_FP32 = 97, 135
FP32_VECTOR_PEAK_TFLOPS = 157.3  # published, packed FP32 FMA


def updates_per_launch(storage: str, nodes: int) -> int:
    """Steps the library fuses per launch: four on the 64 x TY tiles in FP64
    and FP32, two in 16-bit storage."""
    return 2 if storage in ("fp16", "bf16") else 4


def fp32_kernel(n: int) -> str:
    """The kernel of an n x n FP32 lattice's fused launches."""
    return "k_step4<float> (four steps per launch)"


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in STEP_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _counter_value(path, key):
    """A per-launch figure from a committed counter summary, if the counters
    were taken on the current kernel source."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel_source_sha256:\s*(\w+)", txt)
    m_val = re.search(key + r":\s*([0-9.eE+]+)", txt)
    if not (m_hash and m_val) or m_hash.group(1) != kernel_hash():
        return None
    return float(m_val.group(1))


def measured_traffic():
    """HBM bytes per launch of the FP32 step (FETCH_SIZE + WRITE_SIZE)."""
    return _counter_value(TRAFFIC_FILE, "traffic_bytes_per_launch")


def measured_valu():
    """VALU wave instructions per launch of the FP32 step (SQ_INSTS_VALU)."""
    return _counter_value(VALU_FILE, "valu_wave_instructions_per_launch")


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


def cpu_baseline(n, tau, budget_s=15.0):
    """The FP64 oracle on the same cavity, first steps from the same initial
    state, on all host threads, for about budget_s of stepping (after one
    untimed step that starts the thread pool)."""
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


def precision_errors(n=512, steps=20000, tau=0.8):
    """Velocity and strain-rate relative error (Sec. III norm) of FP32, FP16
    and BF16 storage against the FP64 path, Taylor-Green n x n, U0 0.05,
    noise 1e-5, relaxation time tau."""
    import numpy as np
    import torch
    out = {}
    ref = taylor_green_lattice(n, "fp64", tau=tau).step(steps).macroscopic()
    ref = {k: v.cpu().numpy() for k, v in ref.items()}
    den_u = np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2).sum()
    for storage, rounding in (("fp32", "nearest"), ("fp16", "nearest"), ("bf16", "nearest"),
                              ("fp16", "stochastic"), ("bf16", "stochastic")):
        m = taylor_green_lattice(n, storage, tau=tau, rounding=rounding).step(steps).macroscopic()
        m = {k: v.cpu().numpy() for k, v in m.items()}
        eu = np.sqrt((m["ux"] - ref["ux"]) ** 2 + (m["uy"] - ref["uy"]) ** 2).sum() / den_u
        es = np.abs(m["sxx"] - ref["sxx"]).sum() / np.abs(ref["sxx"]).sum()
        key = storage if rounding == "nearest" else f"{storage}_sr"
        out[key] = {"u_rel_err": float(f"{eu:.3e}"), "sxx_rel_err": float(f"{es:.3e}")}
    torch.cuda.synchronize()
    return {"workload": f"taylor_green_{n}x{n}_u0.05_tau{tau}_{steps}steps", "reference": "fp64 GPU path",
            **out}


def adjoint_rollout(n=512, T=2000, every=100):
    """Forward + adjoint of the differentiable rollout (512 x 512 periodic,
    force field N(0, 1e-6^2) seed 4, u0 = 0, Taylor-Green target U0 = 0.02)."""
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
        for _ in range(2):
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
    dt = res["fp32"][0]
    errF = np.abs(res["fp32"][1] - res["fp64"][1]).sum() / np.abs(res["fp64"][1]).sum()
    erru = np.abs(res["fp32"][2] - res["fp64"][2]).sum() / np.abs(res["fp64"][2]).sum()
    return {"workload": f"rollout_{n}x{n}_fp32_T{T}_ckpt{every}", "mlups": round(n * n * T / dt / 1e6, 1),
            "seconds": round(dt, 3), "grad_force_rel_err_vs_fp64": float(f"{errF:.3e}"),
            "grad_u0_rel_err_vs_fp64": float(f"{erru:.3e}")}


def copy_calibration(nbytes=1 << 30):
    """A plain elementwise copy kernel of known size (reads and writes nbytes),
    so that counter runs can scale the step kernel's FETCH_SIZE / WRITE_SIZE
    by what the same counters read for it."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--n", type=int, default=4096, help="cavity size of the headline run")
    ap.add_argument("--only", choices=["fp32", "fp16", "bf16", "fp64", "rollout"], default=None,
                    help="time one storage mode, or the forward + adjoint rollout, only (profiling runs)")
    ap.add_argument("--rounding", choices=["nearest", "stochastic"], default="nearest",
                    help="16-bit rounding of an --only fp16/bf16 run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()
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

    if args.only in ("fp16", "bf16", "fp64"):
        n = 8192 if args.only != "fp64" else 4096
        rounding = args.rounding if args.only != "fp64" else "nearest"
        lat = (taylor_green_lattice(n, args.only, rounding=rounding) if args.only != "fp64"
               else cavity_lattice(n, "fp64")[0])
        grp = updates_per_launch(args.only, n * n)
        dt, dt_main, launches = timed_steps(lat, args.steps, args.warmup, grp)
        mlups = n * n * args.steps / dt / 1e6
        gbs = BYTES_PER_NODE[args.only] * n * n * launches / dt_main / 1e9 if launches else None
        print(json.dumps({"only": args.only, "rounding": rounding, "n": n, "mlups": round(mlups, 1),
                          "updates_per_launch": grp, "moved_gbs": None if gbs is None else round(gbs, 1),
                          "launch_us": round(dt_main / launches * 1e6, 2) if launches else None}))
        return

    n = args.n
    lat, tau = cavity_lattice(n, "fp32")
    grp = updates_per_launch("fp32", n * n)
    if args.steps < grp:
        raise SystemExit(f"--steps must be at least {grp} (one fused launch)")
    dt, dt_main, launches = timed_steps(lat, args.steps, args.warmup, grp)
    mlups = n * n * args.steps / dt / 1e6
    per_launch = dt_main / launches
    moved = BYTES_PER_NODE["fp32"] * n * n / per_launch / 1e9  # HBM bytes the launch moves
    achieved = moved * grp  # algorithmic: 72 B per cell update, grp updates per node
    d = lat.diagnostics()  # raises on a non-finite state
    traffic = measured_traffic() if n == 4096 else None
    valu = measured_valu() if n == 4096 else None
    line = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"cavity_{n}x{n}_re1000_fp32", "nx": n, "ny": n, "tau": round(tau, 6),
                   "lid_u": 0.1, "storage": "fp32", "bc": "halfway bounce-back walls, moving lid"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "kernel": fp32_kernel(n),
                     "launch_us": round(per_launch * 1e6, 2),
                     "updates_per_launch": grp,
                     "alg_bytes_per_update": BYTES_PER_NODE["fp32"],
                     "moved_bytes_per_update": BYTES_PER_NODE["fp32"] / grp,
                     "moved_gbs": round(moved, 1), "moved_frac": round(moved / HBM_PEAK_GBS, 4),
                     "valu": None if valu is None else {
                         "lane_instructions_per_update": round(valu * 64 / (grp * n * n), 1),
                         "achieved_tops": round(valu * 64 / per_launch / 1e12, 2),
                         "peak_tops": round(VALU_PEAK_LANE_OPS / 1e12, 2),
                         "frac": round(valu * 64 / per_launch / VALU_PEAK_LANE_OPS, 4)},
                     "collision": {
                         "ops_per_update": COLLISION_OPS_FP32, "flops_per_update": COLLISION_FLOPS_FP32,
                         "ops_frac": round(COLLISION_OPS_FP32 * grp * n * n / per_launch / VALU_PEAK_LANE_OPS, 4),
                         "achieved_tflops": round(COLLISION_FLOPS_FP32 * grp * n * n / per_launch / 1e12, 2),
                         "fp32_vector_peak_tflops": FP32_VECTOR_PEAK_TFLOPS},
                     "note": f"{grp} steps per launch: the state crosses HBM once per {grp} updates, "
                             "so the algorithmic rate exceeds the single-pass HBM roofline.  The launch "
                             "is bound by VALU issue (valu.frac of 256 CUs x 64 lanes x 2.4 GHz; the "
                             "collision's own operations are collision.ops_frac of it, the rest is the "
                             "recompute ring and staging); its moved bytes run at moved_frac of HBM "
                             "peak (a plain copy reaches 5.07 TB/s)"},
        "mass_drift_rel": float(f"{abs(d[0] / (n * n) - 1.0):.2e}"),
    }
    del lat
    torch.cuda.empty_cache()
    if args.only is None and not args.no_forms:
        # the other grids and Reynolds number of the same cavity throughput study
        sizes = {}
        for ns, re in ((1024, 1000.0), (2048, 1000.0), (4096, 5000.0)):
            ls, _ = cavity_lattice(ns, "fp32", re)
            dts, _, _ = timed_steps(ls, 2100, 300, updates_per_launch("fp32", ns * ns))
            sizes[f"cavity_{ns}x{ns}_re{int(re)}_fp32"] = round(ns * ns * 2100 / dts / 1e6, 1)
            del ls
            torch.cuda.empty_cache()
        line["sizes"] = sizes
    if args.only is None and not args.no_forms:
        forms = {}
        for storage in ("fp16", "bf16"):
            for rounding in ("nearest", "stochastic"):
                l16 = taylor_green_lattice(8192, storage, rounding=rounding)
                g16 = updates_per_launch(storage, 8192 * 8192)
                steps16 = max(10, min(args.steps // 4, 2000))
                steps16 -= steps16 % g16
                dt16, _, launches16 = timed_steps(l16, steps16, max(2, args.warmup // 4), g16)
                m16 = 8192 * 8192 * steps16 / dt16 / 1e6
                moved16 = BYTES_PER_NODE[storage] * 8192 * 8192 / (dt16 / launches16) / 1e9
                alg16 = BYTES_PER_NODE[storage] * m16 / 1e3  # 36 B per cell update
                key = f"{storage}_dev" if rounding == "nearest" else f"{storage}_dev_sr"
                forms[key] = {"workload": "taylor_green_8192x8192", "rounding": rounding,
                              "mlups": round(m16, 1), "updates_per_launch": g16,
                              "alg_gbs": round(alg16, 1), "alg_frac": round(alg16 / HBM_PEAK_GBS, 4),
                              "moved_gbs": round(moved16, 1), "moved_frac": round(moved16 / HBM_PEAK_GBS, 4)}
                del l16
                torch.cuda.empty_cache()
        forms["error_vs_fp64"] = precision_errors()
        forms["error_vs_fp64_tau0.55"] = precision_errors(tau=0.55)
        forms["fwd_adjoint"] = adjoint_rollout()
        line["forms"] = forms
    if args.only is None and not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(n, tau)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
