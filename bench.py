#!/usr/bin/env python3
"""Benchmark of the CTMRG environment hot path on one MI355X.

Workload: the transverse-field Ising iPEPS of the precision-form study --
checkerboard unit cell [[A, B], [B, A]], bond dimension D = 6, environment
chi = 72 (enlarged corners of n = chi D^2 = 2592), FP64.  A step is one
CTMRG iteration (left, up, right, down moves over both columns/rows: 8
moves, 16 projector problems).  Inputs are seeded synthetic tensors
(N(0,1) sites; positive ket/bra-symmetric random boundary), resident in HBM
before timing.  The input boundary is prepared by --prep untimed CTMRG
iterations from the random start, so that the timed moves run in the regime
of the full update, whose environment is always warm-started from the
previous one; then --warmup untimed and --steps timed iterations.

Prints one JSON line with the moves/s value, the contraction kernel's
roofline (algorithmic flops over HIP-event-timed launches) and the CPU
oracle timed on a bounded sample of the same moves.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = ("CTMRG moves/s + MFMA TFLOP/s at D=6 χ=72; time-to-1e-6 energy, "
          "recycled vs plain")
FP64_PEAK_TFLOPS = 78.6
HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(HERE, "profiles", "tgemm_f64_kernel_ctmrg_D6_chi72_traffic.txt")
KERNEL_SRC = os.path.join(HERE, "paper_1411_0391_amd", "csrc", "tgemm.hip")


def measured_traffic():
    """HBM bytes per contraction-kernel launch from the committed rocprofv3
    counter summary, or None when the kernel source has changed since the
    counters were taken (or no summary exists)."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    with open(KERNEL_SRC, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if vals.get("kernel_source_sha256") != sha or "hbm_bytes_per_launch" not in vals:
        return None
    return float(vals["hbm_bytes_per_launch"])


def settled_time(points, ref, rtol):
    """(settled, first) for a run's measurements `points` = [(t, value), ...]
    in time order: `settled` is the time of the first measurement from which
    every later one lies within rtol |ref| of ref, `first` the time of the
    first one within it; None where there is none."""
    near = [abs(v - ref) <= rtol * abs(ref) for _, v in points]
    first = next((t for (t, _), ok in zip(points, near) if ok), None)
    settled = None
    for (t, _), ok in zip(reversed(points), reversed(near)):
        if not ok:
            break
        settled = t
    return settled, first


def copy_calibration(mib):
    """A plain device-to-device copy of known size, run under the HBM byte
    counters to scale them."""
    import torch
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "copies": 3}),
          flush=True)


def cpu_baseline(sites, C, T, chi, cell, moves):
    """The oracle's left move on the same inputs, timed on all host cores."""
    import numpy as np
    from oracle import ctmrg as octm
    ocell = octm.Cell(2, 2, cell)
    t0 = time.perf_counter()
    for x in range(moves):
        C, T, _ = octm.left_move(ocell, sites, C, T, x % 2, chi)
    dt = time.perf_counter() - t0
    return moves / dt, dt


def run_chain(args):
    """The 1D workload: two-site iMPS, chi = 16, J = h = 1, dt = 0.01, 2000
    steps from seeded N(0,1) tensors, plain (environment every step) and
    recycled (an environment step every 20 steps, its gauge fixed by
    --chain-gauge: direct, Sec. III B 1, or iterative, Sec. III B 2);
    energy against -4/pi."""
    import math
    import numpy as np
    import torch
    import paper_1411_0391_amd as tn
    import tninputs
    chi, nsteps, n_re = 16, args.chain_steps, 20
    build = tn.TN_RECYCLE_BUILD_DIRECT if args.chain_gauge == "direct" else tn.TN_RECYCLE_BUILD
    ga, _, gb, _ = tninputs.imps_two_site(0, chi)
    A0 = np.stack([ga / np.linalg.norm(ga), gb / np.linalg.norm(gb)])
    ctx = tn.Context()
    out = {"metric": "1D iTEBD step time and energy, recycled vs plain", "unit": "ms/step",
           "config": {"workload": f"TFIM chain, two-site iMPS, chi={chi}, J=h=1, dt=0.01, "
                                  f"{nsteps} steps, N_Re={n_re}, {args.chain_gauge} gauge fix",
                      "chi": chi, "steps": nsteps},
           "data": "synthetic", "dtype": "f64", "n_gpus": 1}
    exact = -4.0 / math.pi
    for label, recyc in (("plain", False), ("recycled", True)):
        A = torch.from_numpy(A0.copy()).to("cuda")
        env = ctx.env1d(chi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e = None
        for step in range(nsteps):
            last = step == nsteps - 1
            if not recyc:
                _, e1, _ = ctx.itebd_step(A, 1.0, 1.0, 0.01, env, energy=last)
            elif step % n_re == 0:
                _, e1, _ = ctx.itebd_step(A, 1.0, 1.0, 0.01, env, mode=build, energy=last)
            else:
                _, e1, _ = ctx.itebd_step(A, 1.0, 1.0, 0.01, env, mode=tn.TN_RECYCLE_APPLY,
                                          energy=last)
            if last:
                e = e1
            if step % 500 == 499:
                print(f"[bench] chain {label} step {step + 1}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[label] = {"ms_per_step": round(1e3 * dt / nsteps, 4), "seconds": round(dt, 3),
                      "energy": e, "error_vs_exact": abs(e - exact)}
    out["value"] = out["recycled"]["ms_per_step"]
    out["speedup_recycled_over_plain"] = round(out["plain"]["seconds"] /
                                               out["recycled"]["seconds"], 3)
    print(json.dumps(out), flush=True)


def run_classical(args):
    """The classical workload (Sec. I): the partition function of the 2D
    Ising model at inverse temperature --cl-beta by the power method on the
    row transfer matrix with a two-site iMPS, chi = --cl-chi, from seeded
    N(0,1) tensors.  Plain (environment every step), recycled (N_Re =
    --cl-nre after 20 plain steps) and the limit N_Re -> infinity (20 plain steps,
    then an environment step and the dominant eigenvector of its
    renormalized gate, repeated); the environment steps fix the gauge by
    --cl-gauge (direct, Sec. III B 1, or iterative, Sec. III B 2).  ln Z per site is measured every 20 steps
    (every environment step of the limit run).  The plain run goes on until
    ln Z changes by less than 1e-13 over 100 steps; its value is the
    reference, and time-to-1e-10 is the wall time to the first measurement
    from which every later one stays within 1e-10 (relative) of it (a run
    ends once its last five are); the first measurement within 1e-10 is
    reported beside it.  Onsager's exact value is reported
    beside it (finite chi near the critical point leaves a small bias)."""
    import numpy as np
    import torch
    import paper_1411_0391_amd as tn
    import tninputs
    beta, chi, n_re, warm = args.cl_beta, args.cl_chi, args.cl_nre, 20
    build = tn.TN_RECYCLE_BUILD_DIRECT if args.cl_gauge == "direct" else tn.TN_RECYCLE_BUILD
    ga, _, gb, _ = tninputs.imps_two_site(0, chi)
    A0 = np.stack([ga / np.linalg.norm(ga), gb / np.linalg.norm(gb)])
    ctx = tn.Context()
    out = {"metric": "time to ln Z within 1e-10, 2D classical Ising power method, recycled vs plain",
           "unit": "s", "higher_is_better": False,
           "config": {"workload": f"2D classical Ising partition function, iMPS power method on the "
                                  f"row transfer matrix, beta={beta}, chi={chi}, N_Re={n_re}, "
                                  f"N_warm={warm}, {args.cl_gauge} gauge fix", "beta": beta,
                      "chi": chi},
           "data": "synthetic", "dtype": "f64", "n_gpus": 1}

    def run(label, kind, ref=None, max_steps=20000):
        A = torch.from_numpy(A0.copy()).to("cuda")
        env = ctx.env1d(chi)
        hist, t_hit, step, envs = [], None, 0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while step < max_steps:
            if kind == "limit" and step >= warm:
                ctx.ising2d_tm_step(A, beta, env, mode=build)
                _, lz, rc = ctx.ising2d_tm_step(A, beta, env, mode=tn.TN_RECYCLE_LIMIT, lnz=True)
                step += n_re
                envs += 1
            else:
                meas = step % n_re == n_re - 1
                if kind == "plain" or step < warm:
                    mode = tn.TN_PLAIN
                else:
                    mode = build if (step - warm) % n_re == 0 else tn.TN_RECYCLE_APPLY
                _, lz, _ = ctx.ising2d_tm_step(A, beta, env, mode=mode, lnz=meas)
                envs += mode != tn.TN_RECYCLE_APPLY
                step += 1
                if not meas:
                    continue
            t = time.perf_counter() - t0
            hist.append((step, t, lz))
            print(f"[bench] classical {label} step {step} ln Z {lz:.15f} t {t:.2f}s",
                  file=sys.stderr, flush=True)
            if ref is not None and t_hit is None and abs(lz - ref) <= 1e-10 * abs(ref):
                t_hit = t
            if ref is None and len(hist) > 5 and abs(lz - hist[-6][2]) < 1e-13 * abs(lz):
                break
            if (ref is not None and step >= 100 and len(hist) >= 5
                    and all(abs(h[2] - ref) <= 1e-10 * abs(ref) for h in hist[-5:])):
                break
        print(f"[bench] classical {label}: {step} steps, ln Z {hist[-1][2]:.15f}",
              file=sys.stderr, flush=True)
        settled = None
        if ref is not None:
            settled, _ = settled_time([(t, v) for _, t, v in hist], ref, 1e-10)
        return {"steps": step, "environment_steps": envs, "seconds": round(hist[-1][1], 4),
                "ln_z": hist[-1][2], "time_to_1e-10": settled, "first_within_1e-10": t_hit}

    plain = run("plain", "plain")
    ref = plain["ln_z"]
    cap = 4 * plain["steps"]
    plain = run("plain", "plain", ref, cap)
    rec = run("recycled", "recycled", ref, cap)
    lim = run("limit", "limit", ref, cap)
    exact = None
    try:
        sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests"))
        import pins
        exact = pins.onsager_free_energy(beta)
    except ImportError:
        pass
    out.update({"ln_z_ref": ref, "ln_z_onsager": exact, "plain": plain, "recycled": rec,
                "limit": lim, "value": rec["time_to_1e-10"]})
    if plain["time_to_1e-10"] and rec["time_to_1e-10"]:
        out["speedup_recycled_over_plain"] = round(plain["time_to_1e-10"] /
                                                   rec["time_to_1e-10"], 3)
    if plain["time_to_1e-10"] and lim["time_to_1e-10"]:
        out["speedup_limit_over_plain"] = round(plain["time_to_1e-10"] / lim["time_to_1e-10"], 3)
    print(json.dumps(out), flush=True)


def run_mz_sweep(args):
    """Simple update against full update (Sec. VI D, Fig. 26): the
    magnetisation m_z = |<sz>| of the one-site iPEPS (the paper's cell),
    D = 2, chi = 16, dt = 0.01, over a range of fields.  Per field: the
    simple update for --mz-su-steps steps from the seeded near-product
    state, then the full update with recycling (N_Re = 20 after 20 plain
    steps) for --mz-fu-steps steps from the simple-update state; m_z and E
    from the CTMRG environment converged to 1e-10 (chi = 16)."""
    import numpy as np
    import torch
    import paper_1411_0391_amd as tn
    from paper_1411_0391_amd import driver
    import tninputs
    D, chi, dt = 2, 16, 0.01
    Lx, Ly, cell = tninputs.SINGLE_SITE
    cell = list(cell)
    fields = [float(x) for x in args.mz_fields.split(",")]
    A0 = np.stack([a / np.linalg.norm(a) for a in tninputs.ipeps_near_product(0, 1, D)])
    C0, T0 = tninputs.ctm_env(1, 1, chi, D, positive=True)
    ctx = tn.Context()
    sz = np.diag([1.0, -1.0])

    def measure(sites, h):
        C = torch.from_numpy(C0.copy()).to("cuda")
        T = torch.from_numpy(T0.copy()).to("cuda")
        _, it, delta = ctx.ctmrg_iterate(Lx, Ly, sites, cell, C, T, 200, 1e-10)
        e = ctx.ipeps_energy(Lx, Ly, sites, cell, C, T, 1.0, h)
        r1 = ctx.ipeps_rdms(Lx, Ly, sites, cell, C, T)[0].cpu().numpy()
        return abs(float(np.trace(r1[0] @ sz))), e, delta

    rows = []
    t0 = time.perf_counter()
    for h in fields:
        su = driver.simple_update(ctx, Lx, Ly, cell, torch.from_numpy(A0.copy()).to("cuda"), 1.0,
                                  h, dt, args.mz_su_steps)
        m_su, e_su, d_su = measure(su, h)
        C = torch.from_numpy(C0.copy()).to("cuda")
        T = torch.from_numpy(T0.copy()).to("cuda")
        fu, _ = driver.full_update(ctx, Lx, Ly, cell, su.clone(), C, T, 1.0, h, dt,
                                   args.mz_fu_steps, n_re=20, n_warm=20, min_fidelity=1 - 1e-3)
        m_fu, e_fu, d_fu = measure(fu, h)
        rows.append({"h": h, "mz_su": m_su, "mz_fu": m_fu, "E_su": e_su, "E_fu": e_fu,
                     "ctm_delta": max(d_su, d_fu)})
        print(f"[bench] mz h={h}: SU m_z {m_su:.6f} E {e_su:.8f} | FU m_z {m_fu:.6f} "
              f"E {e_fu:.8f} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    out = {"metric": "m_z(h), simple update vs full update (one-site iPEPS)", "unit": "m_z",
           "config": {"workload": f"TFIM one-site iPEPS, D={D}, chi={chi}, dt={dt}, "
                                  f"SU {args.mz_su_steps} steps, then FU (N_Re=20) "
                                  f"{args.mz_fu_steps} steps", "D": D, "chi": chi},
           "data": "synthetic", "dtype": "f64", "n_gpus": 1, "rows": rows,
           "seconds": round(time.perf_counter() - t0, 2)}
    print(json.dumps(out), flush=True)


def run_full_update(args):
    """The 2D full-update workload: checkerboard (or --fu-cell one-site, the
    paper's scheme with averaged links), D = --fu-D (4), chi = --fu-chi (32),
    J = 1, h = 3.0, dt = 0.01, CTMRG tolerance 1e-10, from seeded N(0,1)
    sites and the positive seeded boundary.  The plain run (environment every step)
    goes on until its energy changes by less than --fu-conv (relative) over
    100 steps, or --fu-steps steps; its last energy is E_ref.  The recycled
    run (N_Re = --fu-nre after --fu-warm plain steps; an environment step is
    recycled only when its gauge fix reaches F >= 1 - 1e-3) covers the same
    number of steps.  Time-to-1e-6: wall time from the start of a run to the
    first environment step from which every later one stays within 1e-6
    (relative) of E_ref; a recycled run can overshoot E_ref and return, so the
    first step within 1e-6 is reported beside it but is not the figure."""
    import numpy as np
    import torch
    import paper_1411_0391_amd as tn
    from paper_1411_0391_amd import driver
    import tninputs
    D, chi = args.fu_D, args.fu_chi
    one_site = args.fu_cell == "one-site"
    Lx, Ly, cell = tninputs.SINGLE_SITE if one_site else tninputs.CHECKERBOARD
    cell = list(cell)
    nsite = 1 if one_site else 2
    if args.fu_start == "random":
        A0 = np.stack(tninputs.ipeps_sites(0, nsite, D))
        start = "N(0,1) site tensors of bond D from seed 0"
    else:
        A0 = np.stack(tninputs.ipeps_near_product(0, nsite, D))
        start = "seeded N(0,1) product state plus 1e-2 of N(0,1) bond-D tensors"
    C0, T0 = tninputs.ctm_env(1, Lx * Ly, chi, D, positive=True)
    ctx = tn.Context()
    if args.fu_start == "su":
        # the product start evolved by the simple update (untimed)
        A0 = driver.simple_update(ctx, Lx, Ly, cell, torch.from_numpy(A0.copy()).to("cuda"),
                                  1.0, 3.0, 0.01, args.fu_su_steps).cpu().numpy()
        start += f", then {args.fu_su_steps} simple-update steps (untimed)"
    runs, info_all = {}, {}
    nsteps = args.fu_steps
    for label, n_re, n_warm in (("plain", 1, 0), ("recycled", args.fu_nre, args.fu_warm)):
        C = torch.from_numpy(C0.copy()).to("cuda")
        T = torch.from_numpy(T0.copy()).to("cuda")
        ctx.clear_cache()
        energies, infos = {}, []

        def cb(step, info, label=label, energies=energies, infos=infos):
            energies[step + 1] = info["energy"]
            infos.append(info)
            if label == "plain" or step % 20 == 0 or info["recycled"]:
                print(f"[bench] fu {label} step {step + 1} E {info['energy']:.12f} "
                      f"recycled {info['recycled']} F {info['fidelity']} "
                      f"ctm {info['ctm_iters']} als {info['als_passes']} "
                      f"t {info['seconds']:.1f}s", file=sys.stderr, flush=True)
            if label == "plain" and step + 1 > 100:
                e, e0 = info["energy"], energies[step + 1 - 100]
                return abs(e - e0) < args.fu_conv * abs(e)
            return False

        _, log = driver.full_update(ctx, Lx, Ly, cell, torch.from_numpy(A0.copy()).to("cuda"),
                                    C, T, 1.0, 3.0, 0.01, nsteps, n_re=n_re, n_warm=n_warm,
                                    min_fidelity=1 - 1e-3, callback=cb)
        runs[label] = log
        info_all[label] = infos
        if label == "plain":
            nsteps = log[-1][0]
    e_ref = runs["plain"][-1][1]
    plain_conv = False
    if len(runs["plain"]) > 100:
        plain_conv = abs(runs["plain"][-1][1] - runs["plain"][-101][1]) < args.fu_conv * abs(e_ref)
    out = {"metric": "time-to-1e-6 energy, recycled vs plain (2D full update)", "unit": "s",
           "higher_is_better": False,
           "config": {"workload": f"TFIM iPEPS full update, {args.fu_cell} cell, D={D}, "
                                  f"chi={chi}, h=3.0, dt=0.01, CTMRG tol 1e-10", "D": D,
                      "chi": chi, "cell": args.fu_cell,
                      "steps": nsteps, "N_Re": args.fu_nre, "N_warm": args.fu_warm,
                      "min_fidelity": 1 - 1e-3, "start": start},
           "data": "synthetic", "dtype": "f64", "n_gpus": 1,
           "E_ref": e_ref, "E_ref_converged": plain_conv,
           "E_ref_definition": f"plain run's energy per site once it changes by less than "
                               f"{args.fu_conv:g} (relative) over 100 steps "
                               f"(or after {args.fu_steps} steps)"}
    for label, log in runs.items():
        hit, first = settled_time([(t, e) for _, e, t, *_ in log], e_ref, 1e-6)
        recycled = [i for i in info_all[label] if i["recycled"]]
        fids = [i["fidelity"] for i in info_all[label] if i["fidelity"] is not None]
        out[label] = {"seconds": round(log[-1][2], 3), "env_steps": len(log),
                      "recycled_env_steps": len(recycled), "final_energy": log[-1][1],
                      "time_to_1e-6": hit, "first_within_1e-6": first,
                      "min_fidelity_seen": min(fids) if fids else None,
                      "ctm_iters_mean": float(np.mean([i["ctm_iters"] for i in info_all[label]]))}
    rp, rr = out["plain"]["time_to_1e-6"], out["recycled"]["time_to_1e-6"]
    out["value"] = rr
    out["speedup_recycled_over_plain"] = round(rp / rr, 3) if (rp and rr) else None
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prep", type=int, default=None,
                    help="untimed CTMRG iterations that prepare the input boundary "
                         "(default: iterate until delta < --prep-delta)")
    ap.add_argument("--prep-delta", type=float, default=1e-7,
                    help="prepare the input boundary to this CTMRG delta (at most 100 "
                         "iterations)")
    ap.add_argument("--D", type=int, default=6)
    ap.add_argument("--chi", type=int, default=72)
    ap.add_argument("--cpu-moves", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precision", choices=("fp64", "fp32", "bf16"), default="fp64",
                    help="bulk precision of the contractions (the factorisations stay FP64)")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (counter calibration)")
    ap.add_argument("--chain", action="store_true", help="run the 1D workload instead")
    ap.add_argument("--chain-steps", type=int, default=2000)
    ap.add_argument("--chain-gauge", choices=["direct", "iterative"], default="direct",
                    help="gauge fix of the chain's recycling builds")
    ap.add_argument("--mz", action="store_true",
                    help="m_z(h) of the simple and the full update (one-site iPEPS)")
    ap.add_argument("--mz-fields", default="2.5,2.8,2.9,3.0,3.05,3.1,3.2,3.3,3.5")
    ap.add_argument("--mz-su-steps", type=int, default=1000)
    ap.add_argument("--mz-fu-steps", type=int, default=600)
    ap.add_argument("--classical", action="store_true",
                    help="the classical 2D Ising partition function (power method, recycling)")
    ap.add_argument("--cl-beta", type=float, default=0.42)
    ap.add_argument("--cl-chi", type=int, default=16)
    ap.add_argument("--cl-gauge", choices=["direct", "iterative"], default="direct",
                    help="gauge fix of the recycling's environment steps")
    ap.add_argument("--cl-nre", type=int, default=20,
                    help="N_Re of the recycled power method")
    ap.add_argument("--fu", action="store_true",
                    help="run the 2D full-update time-to-1e-6 workload instead")
    ap.add_argument("--fu-steps", type=int, default=1500,
                    help="step cap of the plain full-update run")
    ap.add_argument("--fu-warm", type=int, default=20)
    ap.add_argument("--fu-nre", type=int, default=20)
    ap.add_argument("--fu-cell", choices=("checkerboard", "one-site"), default="checkerboard",
                    help="unit cell of the full-update workload (one-site: the paper's scheme)")
    ap.add_argument("--fu-D", type=int, default=4)
    ap.add_argument("--fu-chi", type=int, default=32)
    ap.add_argument("--fu-su-steps", type=int, default=300,
                    help="simple-update steps before the full update with --fu-start su")
    ap.add_argument("--fu-start", choices=("random", "product", "su"), default="random",
                    help="start of the full update: N(0,1) bond-D tensors, a random "
                         "product state with a 1e-2 bond-D part, or that state after "
                         "--fu-su-steps simple-update steps")
    ap.add_argument("--fu-conv", type=float, default=1e-9,
                    help="plain run ends when E changes by less than this over 100 steps")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the method's environment "
              "computation is single-device here); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibrate:
        copy_calibration(args.copy_calibrate)
        return
    if args.chain:
        run_chain(args)
        return
    if args.fu:
        run_full_update(args)
        return
    if args.classical:
        run_classical(args)
        return
    if args.mz:
        run_mz_sweep(args)
        return

    import numpy as np
    import torch

    import paper_1411_0391_amd as tn
    import tninputs

    D, chi = args.D, args.chi
    Lx, Ly, cell = tninputs.CHECKERBOARD
    cell = list(cell)
    sites_h = tninputs.ipeps_sites(0, 2, D)
    C_h, T_h = tninputs.ctm_env(1, Lx * Ly, chi, D, positive=True)
    dev = torch.device("cuda:0")
    sites = torch.from_numpy(np.stack(sites_h)).to(dev)
    C = torch.from_numpy(C_h).to(dev)
    T = torch.from_numpy(T_h).to(dev)
    ctx = tn.Context()
    moves_per_step = 4 * Lx
    print(f"[bench] D={D} chi={chi} n={chi * D * D} warmup {args.warmup} steps {args.steps}",
          file=sys.stderr, flush=True)
    if args.prep is not None:
        for w in range(args.prep):
            ctx.ctmrg_moves(Lx, Ly, sites, cell, C, T, moves_per_step, 0)
        prep = f"boundary after {args.prep} CTMRG iterations from a seeded random start"
    else:
        # a boundary at a fixed convergence level, so that the timed work (the
        # subspace iterations per projector follow how much the boundary still
        # moves) does not depend on how it was prepared
        _, pit, pdelta = ctx.ctmrg_iterate(Lx, Ly, sites, cell, C, T, 100, args.prep_delta)
        prep = (f"boundary converged to CTMRG delta {pdelta:.2e} (target {args.prep_delta:g}, "
                f"{pit} iterations from a seeded random start)")
    print(f"[bench] input: {prep}", file=sys.stderr, flush=True)
    prec = args.precision
    C_prep, T_prep = C.clone(), T.clone()
    for w in range(args.warmup):
        ctx.ctmrg_moves(Lx, Ly, sites, cell, C, T, moves_per_step, 0, precision=prec)
        print(f"[bench] warmup step {w + 1} done", file=sys.stderr, flush=True)
    C_bench, T_bench = C.detach().cpu().numpy(), T.detach().cpu().numpy()
    ctx.prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ctx.ctmrg_moves(Lx, Ly, sites, cell, C, T, moves_per_step, 0, precision=prec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.prof_read()
    ctx.prof_enable(False)
    elapsed = t1 - t0
    moves = args.steps * moves_per_step
    value = moves / elapsed
    avg_ms = prof["gemm_ms"] / max(1, prof["gemm_launches"])
    flops_per_launch = prof["gemm_flops"] / max(1, prof["gemm_launches"])
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f}s; gemm {prof['gemm_ms']:.1f} ms "
          f"over {prof['gemm_launches']} launches; svd iters/call "
          f"{prof['svd_iters'] / max(1, prof['svd_calls']):.2f}", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"TFIM iPEPS CTMRG iteration (8 moves), checkerboard, D={D}, "
                               f"chi={chi}, FP64", "D": D, "chi": chi, "cell": "2x2 checkerboard",
                   "moves_per_step": moves_per_step,
                   "input": prep},
        "roofline": {"bound": "mfma", "kernel": "tgemm_f64_kernel",
                     "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": measured_traffic(),
                     "avg_launch_ms": round(avg_ms, 5), "launches": prof["gemm_launches"],
                     "flops_per_launch": flops_per_launch,
                     "algorithmic_bytes_per_launch":
                         prof["gemm_bytes"] / max(1, prof["gemm_launches"])},
        "step_mfma_tflops": round(prof["gemm_flops"] / elapsed / 1e12, 3),
        "svd_iters_per_projector": round(prof["svd_iters"] / max(1, prof["svd_calls"]), 3),
        "svd_at_cap": prof["svd_unconverged"],
        "jacobi_sweeps": prof["jacobi_sweeps"],
    }
    if prec != "fp64":
        # the precision form's energy against the FP64 one: both converge from
        # the prepared boundary to delta < 1e-10, the reduced form with its
        # bulk phase first and at least 5 FP64 iterations after it
        res = {}
        for pr in ("fp64", prec):
            Cq, Tq = C_prep.clone(), T_prep.clone()
            torch.cuda.synchronize()
            tq = time.perf_counter()
            _, it, de = ctx.ctmrg_iterate(Lx, Ly, sites, cell, Cq, Tq, 200, 1e-10, precision=pr,
                                          n_polish=5)
            torch.cuda.synchronize()
            res[pr] = (ctx.ipeps_energy(Lx, Ly, sites, cell, Cq, Tq, 1.0, 3.0), it, de,
                       time.perf_counter() - tq)
        e64, ep = res["fp64"][0], res[prec][0]
        out["precision_form"] = {
            "bulk": prec, "energy_fp64": e64, "energy": ep,
            "energy_rel_error": abs(ep - e64) / abs(e64),
            "iterations_fp64": res["fp64"][1], "iterations": res[prec][1],
            "seconds_to_1e-10_fp64": round(res["fp64"][3], 3),
            "seconds_to_1e-10": round(res[prec][3], 3)}
        out["dtype"] = f"{prec} bulk, f64 factorisations"
        out["config"]["workload"] += f" ({prec} bulk contractions)"
        out["roofline"]["kernel"] = f"tgemm_f64_kernel and tgemm_lp_kernel ({prec})"
        out["roofline"]["note"] = ("averaged over the FP64 and the reduced-precision "
                                   "contractions against the FP64 peak")
    if not args.no_cpu:
        try:
            from threadpoolctl import threadpool_info
            ncores = max(int(i.get("num_threads", 1)) for i in threadpool_info()) or 1
        except Exception:  # no BLAS pool reported: count the host cores
            ncores = os.cpu_count() or 1
        rate, dt = cpu_baseline(sites_h, C_bench, T_bench, chi, cell, args.cpu_moves)
        out["cpu_baseline"] = {"value": round(rate, 5), "unit": "moves/s", "cores": ncores,
                               "kind": "oracle",
                               "sample": f"{args.cpu_moves} left moves of the same workload "
                                         f"from the warmed boundary ({dt:.1f} s)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
