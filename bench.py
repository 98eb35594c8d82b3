#!/usr/bin/env python3
"""Benchmark of the IUGKP particle step on one MI355X.

Workload: the 2D gray square cavity, 256 x 256 uniform cells, hot top wall
T = 1.01, other walls 0.99, constant relaxation time at Kn = 0.01, 0.1, 1 and
10, 1e7 particles per iteration, inexact-Newton diffusion acceleration (FP64
CG, tol 1e-10), int64 fixed-point tallies, face (heat-flux) tallies every
iteration.  Inputs are synthetic and seeded (seed 0).

One step = one full iteration of the hot path for each of the four Kn
problems: emitter split, sampling + flight + tallies, macroscopic update,
Newton CG, residual.  The four problems are independent: each solver has a
stream of its own and the timed steps run through iugkp_step_group, which
enqueues a problem's next iteration as soon as its previous one is done, so
one problem's Newton CG (a few tens of workgroups) overlaps the others'
particle steps.  Printed: one JSON line
with flights/s over the timed (concurrent) steps; per-Kn breakdown and the
roofline of the dominant kernel from a pass of the same steps one problem at
a time (HIP events on each solver's stream); time-to-steady at residual 1e-6 (common
random numbers, faces tallied on the output iteration), the batched solver
against sequential solves, the adjoint gradient, the 40-band non-gray
two-material problem and the CPU oracle baseline on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

KNS = (0.01, 0.1, 1.0, 10.0)
N_SIDE = 256
PARTICLES = 10_000_000
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tts", action="store_true", help="skip time-to-steady")
    ap.add_argument("--batch", type=int, default=256,
                    help="instances of the batched vs sequential comparison (0: skip)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint gradient timing")
    ap.add_argument("--no-c0", action="store_true", help="skip the 1D slab time-to-steady")
    ap.add_argument("--no-c2-gray", action="store_true",
                    help="skip the 512^2 gray two-material throughput")
    ap.add_argument("--no-nongray", action="store_true", help="skip the 40-band timing")
    ap.add_argument("--no-expected", action="store_true",
                    help="skip the expected-value estimator comparison")
    ap.add_argument("--expected-only", action="store_true",
                    help="only the expected-value comparison (its own JSON line; for profiling)")
    ap.add_argument("--no-persistent", action="store_true",
                    help="skip the persistent-particle timing")
    ap.add_argument("--persistent-only", action="store_true",
                    help="only the persistent-particle timing (its own JSON line; for profiling)")
    ap.add_argument("--nongray-only", action="store_true",
                    help="only the 40-band timing (printed as its own JSON line; for profiling)")
    ap.add_argument("--c2-gray-only", action="store_true",
                    help="only the 512x512 two-material gray timing (its own JSON line; for profiling)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched vs sequential comparison (its own JSON line)")
    ap.add_argument("--forms", default=None,
                    help="(with --profile-pass) JSON {kn: particle-step form} to run the problems in")
    ap.add_argument("--profile-pass", action="store_true",
                    help="only the kernel pass that the counter collection profiles")
    ap.add_argument("--no-counters", action="store_true",
                    help="skip the rocprofv3 counter passes (HBM bytes, atomics, occupancy)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 256 MiB buffer three times (scales rocprofv3 FETCH_SIZE / "
                         "WRITE_SIZE to bytes) and exit")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000,
                    help="particles per iteration in the CPU oracle sample")
    return ap.parse_args()


def march_bytes(flights, crossings, segments, n_emit, has_null):
    """Algorithmic bytes of the particle step: 8 B read-modify-write per face
    crossing and per final deposit/absorption, the emitter split (12 B per
    emitter), and per null segment the relaxation-ratio gather plus the W tally
    (16 B)."""
    b = 8 * (crossings + flights) + 12 * n_emit
    if has_null:
        b += 16 * segments
    return b


def cg_bytes(cg_iters, n_cells):
    """Per CG iteration: operator application reading r, p_old and three
    coefficient arrays and writing p and Ap, then x, r updates reading x, p, r,
    Ap and writing x, r: 13 doubles per cell."""
    return 13 * 8 * n_cells * cg_iters


MG_LOCAL_MAX = 1024   # levels of at most this many cells stay in LDS


def mgcg_bytes(cg_iters, nx, ny):
    """Per iteration of the multigrid-preconditioned CG, each vector a phase
    reads or writes counted once per cell (a row of the operator as diagonal
    plus two faces): the CG update 12 doubles per fine cell (u, w, p, s, x, r
    and the diagonal read; p, s, x, r and the first sweep written), w = A u 6
    (u, r, row; w); per level spread over the GPU 24 per cell (second
    pre-sweep 6, residual for the restriction 5, corrected post-sweep 7, last
    post-sweep 6) and 3 per aggregate written by the restriction.  The levels
    kept in LDS cost no memory traffic."""
    sizes = []
    while True:
        sizes.append(nx * ny)
        if nx == 1 and ny == 1:
            break
        nx, ny = (nx + 1) // 2, (ny + 1) // 2
    Lg = 0
    while Lg < len(sizes) and sizes[Lg] > MG_LOCAL_MAX:
        Lg += 1
    doubles = 18 * sizes[0] + 24 * sum(sizes[:Lg]) + 3 * sum(sizes[1:Lg + 1])
    return 8 * doubles * cg_iters


def source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hpp", "device_core.hpp", "mgcg.hpp", "iugkp.hip"):
        with open(os.path.join(ROOT, "paper_2506_09465_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(sample):
    """The CPU oracle on a bounded sample of the same step: for each Kn one
    iteration with `sample` particles, once with and once without the Newton
    CG, on one core.  The particle part is scaled to the full particle count;
    the CG part is at full size already."""
    import numpy as np
    from oracle import oracle as O
    from synth import cavity_2d
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import cp_model as cp
    O.build()
    t_total = 0.0
    flights_full = 0
    detail = {}
    for kn in KNS:
        w = cavity_2d(n=N_SIDE, kn=kn, particles=sample, newton=True)
        lam = w.vg * w.tau
        D = np.full(w.n_cells, cp.d_eff(float(lam[0]), w.dx))
        # the Newton-accelerated state: every cell emits after the first iteration
        o = O.Oracle(w, newton=True, diff_x=D, diff_y=D, tally_faces=O.FACES_EVERY,
                     cg_precond=O.PRECOND_MG)
        o.step(2)
        t0 = time.perf_counter()
        o.step(1)
        t_newton = time.perf_counter() - t0
        fl = o.info().flights
        # the same state without the CG: particle part alone
        o_plain = O.Oracle(w, newton=False, tally_faces=O.FACES_EVERY)
        it, d0, E, G = o.info().iter, o.info().d0, o.E(), o.G()
        o_plain.set_state(it, d0, E, G)
        t0 = time.perf_counter()
        o_plain.step(1)
        t_march = time.perf_counter() - t0
        t_cg = max(0.0, t_newton - t_march)
        scale = PARTICLES / sample
        t_full = t_march * scale + t_cg
        t_total += t_full
        flights_full += fl * scale
        detail[str(kn)] = {"s_particles_sampled": round(t_march, 3), "s_cg": round(t_cg, 3),
                           "flights_sampled": fl, "s_full_iteration_est": round(t_full, 2)}
    return {"value": flights_full / t_total, "unit": "flights/s", "cores": 1, "kind": "oracle",
            "sample": f"one iteration per Kn of the 256x256 cavity with {sample} particles "
                      f"(particle time scaled x{PARTICLES // sample} to 1e7) plus the full-size "
                      f"Newton CG, single thread", "detail": detail}


def bench_batch(P, dev, count):
    """Uneven batch of independent cavities (sides 32..256, Kn log-uniform in
    [1e-3, 10], random walls, 1e4..1e6 particles, Newton with the multigrid-
    preconditioned CG, CRN, residual 1e-6):
    the same problems solved one by one through iugkp_solve, then together
    through iugkp_batch_solve.  Both paths do identical work per instance
    (bitwise equal results, same iteration counts and statuses)."""
    import torch
    from synth import batch_workloads
    ws = batch_workloads(count=count)
    kw = dict(rng_mode=P.RNG_CRN, tally_faces=P.FACES_FINAL, max_iters=60, res_tol=1e-6,
              cg_precond=P.PRECOND_MG)
    seq_status = []
    # (the sequential solves take the planner's particle-step form: every
    # instance is a class of its own, and a form search per solve would only
    # add its candidate iterations to the sequential time)
    solvers = [P.Solver(w, device=dev, block_size=256, **kw) for w in ws]
    torch.cuda.synchronize()
    a = time.perf_counter()
    for s in solvers:
        try:
            rc = s.solve()[0]
        except P.IugkpError as e:
            rc = e.code
        seq_status.append(rc)
    torch.cuda.synchronize()
    seq = time.perf_counter() - a
    for s in solvers:
        s.close()
    bs = P.BatchSolver(ws, device=dev, **kw)
    torch.cuda.synchronize()
    a = time.perf_counter()
    rc, outs = bs.solve()
    torch.cuda.synchronize()
    bat = time.perf_counter() - a
    tune_a, tune_c, groups = bs.tuning()
    edges = bs.tile_edges()
    bat_status = [o[3]["status"] for o in outs]
    iters = [o[3]["iters"] for o in outs]
    flights = sum(o[3]["tot_flights"] for o in outs)
    return {"instances": len(ws), "sequential_s": round(seq, 3), "batched_s": round(bat, 3),
            "speedup": round(seq / bat, 3), "same_status": seq_status == bat_status,
            "converged": sum(1 for x in bat_status if x == 0),
            "not_converged": sum(1 for x in bat_status if x == 1),
            "failed": sum(1 for x in bat_status if x < 0),
            "statuses": {str(c): bat_status.count(c) for c in sorted(set(bat_status))},
            "iterations_total": int(sum(iters)), "flights_total": int(flights),
            "batched_flights_per_s": flights / bat,
            "autotuner": {"model_us_per_iteration": round(tune_a, 3),
                          "model_us_per_cell_per_workgroup": round(tune_c, 6),
                          "multigrid_groups_last_replay": {str(int(g)): int((groups == g).sum())
                                                           for g in sorted(set(groups.tolist()))
                                                           if g > 0},
                          "tile_edges": {str(int(e)): int((edges == e).sum())
                                         for e in sorted(set(edges.tolist()))},
                          "note": "group sizes of the multigrid pool chosen before every replay "
                                  "from a fit of the measured job durations; tile edges of the "
                                  "tile march chosen per instance class from the device time per "
                                  "flight of a replay with each (the second and third replays)"},
            "note": "per-instance setup (allocation, Newton operator) excluded from both timings"}


def bench_adjoint(P, dev):
    """The adjoint workload: 256 x 256 cavity at Kn = 0.1 with a Gaussian source,
    squared misfit at 64 random probes; forward CRN solve (Newton, residual
    1e-9) and the backward pass (adjoint to relative change 1e-10) timed
    separately."""
    import torch
    from synth import adjoint_case
    case = adjoint_case(n=N_SIDE, kn=0.1, n_probes=64, particles=PARTICLES)
    w = case.workload
    probes = torch.tensor(case.probes, device=dev)
    target = torch.tensor(case.target, device=dev)
    walls = torch.tensor(case.walls4, device=dev, requires_grad=True)
    src = torch.tensor(w.source, device=dev, requires_grad=True)
    torch.cuda.synchronize()
    a = time.perf_counter()
    T = P.steady_temperature(walls, src, w, max_iters=200, res_tol=1e-9, newton=True)
    loss = ((T[probes] - target) ** 2).sum()
    torch.cuda.synchronize()
    b = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    c = time.perf_counter()
    return {"forward_s": round(b - a, 4), "backward_s": round(c - b, 4),
            "loss": loss.item(), "grad_walls": [round(x, 12) for x in walls.grad.tolist()],
            "grad_source_norm": src.grad.norm().item()}


def tally_roofline(ceil, tallies, launches, ms_launch, bytes_launch, kernel):
    """A particle step's roofline: its algorithmic tally updates (one per face
    crossed, per candidate and per final deposit or absorption) per second
    against the LDS int64-atomic ceiling."""
    t = tallies / launches
    rate = t / (ms_launch / 1e3) if ms_launch else None
    return {"bound": "atomics", "achieved": rate, "peak": ceil["lds_int64_per_s"],
            "unit": "tally atomics/s", "frac": round(rate / ceil["lds_int64_per_s"], 5) if rate else None,
            "traffic": None, "kernel": kernel, "avg_launch_ms": round(ms_launch, 4),
            "algorithmic_atomics_per_launch": int(t), "algorithmic_bytes_per_launch": int(bytes_launch)}


def atomics_ceiling(P):
    """The tally-throughput ceilings a particle step works against: int64
    atomic adds to random words of a 2 MB global array (the size of the
    cavity's tallies) and of a workgroup's LDS array."""
    return {"global_int64_2MB_per_s": P.dev_atomics(False, n_words=262144),
            "lds_int64_per_s": P.dev_atomics(True),
            "note": "int64 atomic adds to random words, every lane of full wavefronts: of a "
                    "2 MB global array, and of a 4096-word LDS array per workgroup"}


def bench_nongray(P, dev, steps, warmup, ceil):
    """The non-gray workload: 512 x 512 two-material square (left half's
    relaxation times 100x the right half's), 40 bands of the sine dispersion
    (Kn 1e-3 .. 10), Gaussian source of width 0.05 L at the centre, 5e7
    particles per iteration.  After `warmup` iterations from t_ref (the
    emission spreads from walls and source) `steps` iterations are timed with
    face tallies every iteration and again without them."""
    import torch
    from synth import nongray_two_material_2d
    w = nongray_two_material_2d()
    s = P.Solver(w, device=dev, tally_faces=P.FACES_EVERY)
    s.step(warmup, faces=False)
    out = {"workload": "2D non-gray two-material 512x512, 40 bands, Gaussian source, "
                       "5e7 particles/iteration", "warmup_iterations": warmup,
           "fixed_point_F": s.stats()["fixed_point_F"]}
    for faces in (True, False):
        a = s.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            assert s.step(1, faces=faces) == 0
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        b = s.stats()
        fl = b["tot_flights"] - a["tot_flights"]
        cr = b["tot_crossings"] - a["tot_crossings"]
        sg = b["tot_segments"] - a["tot_segments"]
        ms_m = (b["ms_march"] - a["ms_march"]) / steps
        mb = march_bytes(fl, cr, sg, b["n_emitters"] * steps, True) / steps
        out["faces_every" if faces else "faces_off"] = {
            "flights_per_s": fl / el, "ms_per_iteration": round(el / steps * 1e3, 3),
            "ms_march": round(ms_m, 3), "flights_per_iter": fl // steps,
            "crossings_per_flight": round(cr / max(fl, 1), 2),
            "segments_per_flight": round(sg / max(fl, 1), 2),
            "march_GBs_algorithmic": round(mb / (ms_m / 1e3) / 1e9, 2) if ms_m else None,
            "roofline": tally_roofline(ceil, cr + sg + fl, steps, ms_m, mb, "march_kernel")}
    s.close()
    return out


def persist_bytes(n, n_null, n_real, crossings):
    """Algorithmic bytes of one persistent move: per particle its kind and
    location (4 B), the state of a null particle (40 B) or the share of a
    resampled one (8 B), the new state (44 B), the W tally (8 B) and for real
    collisions the W^h tally (8 B); 8 B per face crossing tallied."""
    return 48 * n + 40 * n_null + 8 * (n - n_null) + 8 * n + 8 * n_real + 8 * crossings


def bench_persistent(P, dev, steps, ceil, warmup=3):
    """The persistent-particle scheme (Sec. 3.2 steps (1)-(6), fixed
    population) on the 256 x 256 cavity at each Kn with 1e7 particles, face
    tallies every iteration: particle moves per second and the move kernel's
    roofline."""
    import torch
    from synth import cavity_2d
    out = {"workload": "2D gray square cavity 256x256, hot top wall, Kn in {0.01,0.1,1,10}, "
                       "persistent population of 1e7 particles, face tallies every iteration"}
    tot_moves, tot_s, tot_ms, tot_bytes, tot_cr, launches = 0, 0.0, 0.0, 0, 0, 0
    for kn in KNS:
        w = cavity_2d(n=N_SIDE, kn=kn, particles=PARTICLES, newton=False, seed=0)
        s = P.Solver(w, device=dev, scheme=P.SCHEME_PERSISTENT, tally_faces=P.FACES_EVERY)
        s.step(warmup)
        n = s.stats()["segments"]
        t_el, ms, byt, cr = 0.0, 0.0, 0, 0
        for _ in range(steps):
            sh = s.shares()
            n_real0 = int(sh["Nrc"].sum())
            n_wall0 = int(sh["Nb"].sum())
            a = s.stats()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            assert s.step(1) == 0
            torch.cuda.synchronize()
            t_el += time.perf_counter() - t0
            b = s.stats()
            n_real1 = int(s.shares()["Nrc"].sum())
            dcr = b["tot_crossings"] - a["tot_crossings"]
            ms += b["ms_march"] - a["ms_march"]
            byt += persist_bytes(n, n - n_real0 - n_wall0, n_real1, dcr)
            cr += dcr
        s.close()
        out[str(kn)] = {"moves_per_s": n * steps / t_el, "ms_per_iteration": round(t_el / steps * 1e3, 3),
                        "ms_move": round(ms / steps, 3), "crossings_per_move": round(cr / (n * steps), 3),
                        "move_GBs_algorithmic": round(byt / (ms / 1e3) / 1e9, 1)}
        tot_moves += n * steps
        tot_s += t_el
        tot_ms += ms
        tot_bytes += byt
        tot_cr += cr
        launches += steps
    avg_ms = tot_ms / launches
    out["moves_per_s"] = tot_moves / tot_s
    # one end tally per move and one per face crossed, as the emitter scheme's
    # particle step counts them
    out["roofline"] = tally_roofline(ceil, tot_cr + tot_moves, launches, avg_ms,
                                     tot_bytes / launches,
                                     "persist_move_kernel + persist_faces_kernel")
    return out


def bench_expected(P, dev, iters=6, warmup=10):
    """The expected-value estimator against the analog one on the 256 x 256
    cavity at each Kn (1e7 particles, Newton, no face tallies): time per
    iteration, and the steady-state noise of E (RMS over cells of the standard
    deviation of E across FRESH iterations after warm-up); efficiency =
    1 / (noise^2 x time per iteration)."""
    import numpy as np
    import torch
    from synth import cavity_2d
    out = {"workload": "2D gray square cavity 256x256, hot top wall, Kn in {0.01,0.1,1,10}, "
                       "1e7 particles/iteration, Newton, no face tallies; FRESH iterations at "
                       "steady state"}
    for kn in KNS:
        row = {}
        for name, est in (("analog", P.EST_ANALOG), ("expected", P.EST_EXPECTED)):
            w = cavity_2d(n=N_SIDE, kn=kn, particles=PARTICLES, newton=True, seed=0)
            s = P.Solver(w, device=dev, estimator=est, tally_faces=P.FACES_OFF)
            s.step(warmup)
            a = s.stats()
            Es, el = [], 0.0
            for _ in range(iters):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                assert s.step(1) == 0
                torch.cuda.synchronize()
                el += time.perf_counter() - t0
                Es.append(s.state()[2].cpu().numpy())
            b = s.stats()
            s.close()
            Es = np.array(Es)
            noise = float(np.sqrt(np.mean(np.var(Es, axis=0, ddof=1))))
            t_it = el / iters
            row[name] = {"ms_per_iteration": round(t_it * 1e3, 3),
                         "ms_march": round((b["ms_march"] - a["ms_march"]) / iters, 3),
                         "crossings_per_flight": round((b["tot_crossings"] - a["tot_crossings"]) /
                                                       max(1, b["tot_flights"] - a["tot_flights"]), 1),
                         "noise_rms": noise, "efficiency": 1.0 / (noise * noise * t_it)}
        row["efficiency_gain"] = round(row["expected"]["efficiency"] / row["analog"]["efficiency"], 3)
        out[str(kn)] = row
    return out


def host_cpu():
    """The host's CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "usable_cores": usable}


def _oracle_particle_sample(sample, barrier=None, queue=None):
    """One copy of the all-core sample: one face-tallied iteration without the
    Newton CG per Kn of the 256^2 cavity from the seeded temperature field,
    `sample` particles, timed after every copy has set up (barrier); returns
    or queues (flights, seconds)."""
    from oracle import oracle as O
    from synth import cavity_2d, seeded_temperature
    os_ = []
    for kn in KNS:
        w = cavity_2d(n=N_SIDE, kn=kn, particles=sample, newton=False)
        os_.append(O.Oracle(w, newton=False, tally_faces=O.FACES_EVERY,
                            T_init=seeded_temperature(N_SIDE * N_SIDE)))
    if barrier is not None:
        barrier.wait()
    t0 = time.perf_counter()
    for o in os_:
        o.step(1)
    el = time.perf_counter() - t0
    fl = sum(o.info().flights for o in os_)
    if queue is not None:
        queue.put((fl, el))
    return fl, el


def cpu_baseline_all_cores(sample, procs):
    """The unmodified single-thread oracle run as `procs` concurrent copies of
    the same particle-step sample, started together after their set-up: the
    host's aggregate oracle throughput (all copies' flights over the longest
    copy's time)."""
    import multiprocessing as mp
    from oracle import oracle as O
    O.build()
    one = _oracle_particle_sample(sample)              # alone, for the per-core rate
    ctx = mp.get_context("spawn")                      # no fork of a process holding the GPU
    barrier = ctx.Barrier(procs)
    queue = ctx.Queue()
    ps = [ctx.Process(target=_oracle_particle_sample, args=(sample, barrier, queue))
          for _ in range(procs)]
    for p in ps:
        p.start()
    res = [queue.get(timeout=600) for _ in ps]
    for p in ps:
        p.join(timeout=60)
    fl = sum(r[0] for r in res)
    wall = max(r[1] for r in res)
    return {"value": fl / wall, "unit": "flights/s", "cores": procs, "kind": "oracle",
            "single_core_flights_per_s": one[0] / one[1],
            "sample": f"{procs} concurrent copies of the single-thread oracle, each one "
                      f"face-tallied iteration per Kn of the 256x256 cavity without the Newton "
                      f"CG, {sample} particles, from a seeded temperature field, timed together "
                      f"after set-up; value = all copies' flights / the longest copy's time"}


def bench_c0_time_to_steady(P, dev):
    """The 1D slab of 100 cells at Kn = 1 (walls 1.01 / 0.99), 1e5 particles per
    iteration, common random numbers (seed 0), no Newton step, to residual
    1e-6: the GPU solve and the CPU oracle's solve of the same problem (the
    same iterations, bit for bit)."""
    import torch
    from synth import slab_1d
    w = slab_1d(n=100, kn=1.0, particles=100_000, seed=0)
    kw = dict(rng_mode=P.RNG_CRN, tally_faces=P.FACES_FINAL, max_iters=500, res_tol=1e-6)
    P.Solver(w, device=dev, **kw).solve()          # first launches, outside the timing
    s = P.Solver(w, device=dev, **kw)
    torch.cuda.synchronize()
    a = time.perf_counter()
    rc, T, qx, qy, st = s.solve()
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - a
    s.close()
    out = {"workload": "1D gray slab, 100 cells, Kn = 1, walls 1.01/0.99, 1e5 particles per "
                       "iteration, CRN seed 0, no Newton, residual 1e-6",
           "seconds": round(gpu_s, 5), "iterations": st["iters"], "rc": rc,
           "final_res": st["res"], "flights_total": st["tot_flights"],
           "flights_per_s": st["tot_flights"] / gpu_s}
    from oracle import oracle as O
    O.build()
    o = O.Oracle(w, rng_mode=O.CRN, tally_faces=O.FACES_FINAL, max_iters=500, res_tol=1e-6)
    a = time.perf_counter()
    rco, To, _, _ = o.solve()
    cpu_s = time.perf_counter() - a
    out["oracle"] = {"seconds": round(cpu_s, 4), "iterations": o.info().iter, "rc": rco,
                     "cores": 1, "same_T": bool(np.array_equal(To, T.cpu().numpy()))}
    return out


def bench_c2_gray(P, dev, steps, ceil):
    """The 512 x 512 gray two-material square (left half's relaxation time 100x
    the right half's, Kn 0.01 on the right: about 99 of 100 candidate
    collisions in the left half are null), 5e7 particles per iteration, face
    tallies every iteration, no Newton step, from the seeded temperature field
    (every cell emits): four warm-up iterations (the particle-step form
    search: an untimed iteration, then one per form), then `steps` timed."""
    import torch
    from synth import seeded_temperature, two_material_2d
    w = two_material_2d(n=512, kn_right=0.01, ratio=100.0, particles=50_000_000, seed=0)
    s = P.Solver(w, device=dev, tally_faces=P.FACES_EVERY, T_init=seeded_temperature(512 * 512))
    assert s.step(4) == 0
    form, form_ms = s.march_tuning()
    a = s.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    assert s.step(steps) == 0
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    b = s.stats()
    s.close()
    fl = b["tot_flights"] - a["tot_flights"]
    sg = b["tot_segments"] - a["tot_segments"]
    cr = b["tot_crossings"] - a["tot_crossings"]
    ms_m = (b["ms_march"] - a["ms_march"]) / steps
    return {"workload": "2D gray two-material 512x512 (tau_left = 100 tau_right, Kn_right "
                        "0.01), 5e7 particles/iteration, face tallies, no Newton",
            "flights_per_s": fl / el, "ms_per_iteration": round(el / steps * 1e3, 3),
            "ms_march": round(ms_m, 3), "flights_per_iter": fl // steps,
            "segments_per_flight": round(sg / max(fl, 1), 2),
            "crossings_per_flight": round(cr / max(fl, 1), 2),
            "segments_per_s": sg / el, "march_form": form,
            "march_form_ms": {f: (round(v, 3) if v is not None else None)
                              for f, v in form_ms.items()},
            "roofline": tally_roofline(ceil, cr + sg + fl, steps, ms_m,
                                       march_bytes(fl, cr, sg, b["n_emitters"] * steps, True) / steps,
                                       {"stripes": "march_stripes_kernel",
                                        "stripes_pieces": "march_stripes_pieces_kernel"}.get(
                                           form, "march_kernel"))}


def cpu_baseline_nongray():
    """The CPU oracle on a bounded sample of the 40-band problem: the same
    two-material 40-band workload on a 128 x 128 mesh with one particle per
    emitter and band, four iterations from t_ref and then one timed iteration
    with face tallies, on one core."""
    from oracle import oracle as O
    from synth import nongray_two_material_2d
    O.build()
    n = 128
    w = nongray_two_material_2d(n=n, particles=(n * n + 4 * n) * 40)
    o = O.Bands(w, tally_faces=O.FACES_EVERY)
    o.step(4, faces=False)
    t0 = time.perf_counter()
    o.step(1, faces=True)
    el = time.perf_counter() - t0
    i = o.info()
    return {"value": i.flights / el, "unit": "flights/s", "cores": 1, "kind": "oracle",
            "segments_per_s": i.segments / el,
            "sample": "one face-tallied iteration of the two-material 40-band problem on a "
                      "128x128 mesh (1 particle per emitter and band, after 4 iterations from "
                      "t_ref), single thread"}


# kernels of the particle step (between the step's HIP events) and of the Newton CG
PS_KERNELS = ("march_kernel", "stripe_presample_kernel", "march_stripes_kernel",
              "march_stripes_pieces_kernel")
CG_KERNELS = ("mgcg_kernel", "mgcg_band_kernel")
PROFILE_ITERS = 2
# rocprofv3 counter passes (each within one pass's hardware limits: TCC <= 4,
# SQ <= 8, TCP <= 4); FETCH_SIZE and WRITE_SIZE in KiB per dispatch
COUNTER_PASSES = (("FETCH_SIZE",),
                  ("WRITE_SIZE", "TCC_EA0_ATOMIC_sum"),
                  ("SQ_INSTS_LDS", "SQ_WAVES", "MeanOccupancyPerActiveCU",
                   "TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum"))


# a particle-step form as Solver options (the form search keeps the fastest)
FORM_OPTS = {"tiles256": dict(march=1, block_size=256), "tiles512": dict(march=1, block_size=512),
             "stripes": dict(march=2), "stripes_pieces": dict(march=3)}


def profile_pass(forms=None):
    """What collect_counters profiles: a 256 MiB device copy three times (to
    scale FETCH_SIZE / WRITE_SIZE to bytes), then the benchmark's four Kn
    problems one at a time, PROFILE_ITERS iterations each, started from the
    seeded temperature field so that every iteration emits from every cell as
    the benchmark's steady iterations do."""
    import torch
    import paper_2506_09465_amd as P
    from synth import cavity_2d, seeded_temperature
    dev = torch.device("cuda:0")
    n = 256 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    for kn in KNS:
        w = cavity_2d(n=N_SIDE, kn=kn, particles=PARTICLES, newton=True, seed=0)
        # the form the benchmark's search chose, else the planner's (a set
        # block size: no search)
        f = (forms or {}).get(str(kn))
        opts = FORM_OPTS[f] if f in FORM_OPTS else dict(block_size=256)
        s = P.Solver(w, device=dev, tally_faces=P.FACES_EVERY, cg_precond=P.PRECOND_MG,
                     T_init=seeded_temperature(N_SIDE * N_SIDE), **opts)
        assert s.step(PROFILE_ITERS) == 0
        torch.cuda.synchronize()
        s.close()
    print(json.dumps({"profile_pass": "done"}), flush=True)


def _read_counter_csv(root):
    """[(kernel name, grid size, {counter: value})] per dispatch, in dispatch
    order, from every *counter_collection.csv under root."""
    import csv
    import glob
    rows = {}
    for f in glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                d = rows.setdefault(int(r["Dispatch_Id"]),
                                    (r["Kernel_Name"], int(r.get("Grid_Size", 0) or 0), {}))
                d[2][r["Counter_Name"]] = d[2].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [rows[k] for k in sorted(rows)]


def _kernel_is(name, kernels):
    return any(k + "<" in name or k + "(" in name or name.endswith(k) for k in kernels)


def collect_counters(forms=None, timeout_s=240):
    """Run profile_pass under rocprofv3 once per counter pass and reduce the
    per-dispatch counters to per-launch figures of the particle step (all
    its kernels of one iteration) and of the multigrid CG.  Each pass is
    reduced on its own (by kernel name), so the passes need not number their
    dispatches alike."""
    import shutil
    import subprocess
    import tempfile
    prof = shutil.which("rocprofv3") or "/opt/rocm/bin/rocprofv3"
    if not os.path.exists(prof):
        return {"error": "rocprofv3 not found"}
    env = dict(os.environ, TMPDIR="/tmp")
    launches = len(KNS) * PROFILE_ITERS
    groups = {"particle_step": PS_KERNELS, "multigrid_cg": CG_KERNELS}
    tot = {g: {} for g in groups}
    ndisp = {g: 0 for g in groups}
    occ = {g: [] for g in groups}
    copy = {}
    cmds = []
    for counters in COUNTER_PASSES:
        out = tempfile.mkdtemp(prefix="iugkp_pmc_", dir="/tmp")
        cmd = [prof, "--pmc", *counters, "-d", out, "-o", "run", "--output-format", "csv", "--",
               sys.executable, os.path.join(ROOT, "bench.py"), "--profile-pass"]
        if forms:
            cmd += ["--forms", json.dumps(forms)]
        cmds.append(" ".join(["rocprofv3", "--pmc", *counters, "-d", "<dir>", "-o", "run",
                              "--output-format", "csv", "--", "python3", "bench.py",
                              "--profile-pass"] +
                             (["--forms", "'" + json.dumps(forms) + "'"] if forms else [])))
        try:
            r = subprocess.run(cmd, cwd="/tmp", env=env, timeout=timeout_s,
                               stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        except subprocess.TimeoutExpired:
            return {"error": f"counter pass {counters} timed out"}
        rows = _read_counter_csv(out)
        shutil.rmtree(out, ignore_errors=True)
        if not rows:
            return {"error": f"counter pass {counters} produced no data (rc {r.returncode})"}
        # the calibration copies: the three largest copy dispatches
        cp = sorted([d for d in rows if "copyBuffer" in d[0]], key=lambda d: -d[1])[:3]
        for d in cp:
            for k, v in d[2].items():
                copy[k] = copy.get(k, 0.0) + v / len(cp)
        for g, names in groups.items():
            ds = [d for d in rows if _kernel_is(d[0], names)]
            if counters == COUNTER_PASSES[0]:
                ndisp[g] = len(ds)
            for d in ds:
                for k, v in d[2].items():
                    if k == "MeanOccupancyPerActiveCU":
                        occ[g].append(v)
                    else:
                        tot[g][k] = tot[g].get(k, 0.0) + v
    nbytes = 256 * 1024 * 1024
    fk, wk = copy.get("FETCH_SIZE", 0.0), copy.get("WRITE_SIZE", 0.0)
    f_fac = nbytes / (fk * 1024.0) if fk > 0 else None
    w_fac = nbytes / (wk * 1024.0) if wk > 0 else None

    def reduce(g):
        t = tot[g]
        r = {"dispatches": ndisp[g], "launches": launches,
             "fetch_kib": t.get("FETCH_SIZE", 0.0) / launches,
             "write_kib": t.get("WRITE_SIZE", 0.0) / launches,
             "ea_atomic_requests": t.get("TCC_EA0_ATOMIC_sum", 0.0) / launches,
             "tcp_atomic_requests": t.get("TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum", 0.0) / launches,
             "lds_wave_instructions": t.get("SQ_INSTS_LDS", 0.0) / launches,
             "waves": t.get("SQ_WAVES", 0.0) / launches,
             "mean_occupancy_waves_per_active_cu":
                 (sum(occ[g]) / len(occ[g])) if occ[g] else None}
        if f_fac and w_fac:
            r["hbm_bytes"] = (r["fetch_kib"] * f_fac + r["write_kib"] * w_fac) * 1024.0
        return r

    return {"source": "rocprofv3 --pmc, run by this benchmark (profile_pass: the four Kn "
                      f"problems, {PROFILE_ITERS} iterations each, from a seeded temperature "
                      "field)",
            "commands": cmds, "fetch_factor": f_fac, "write_factor": w_fac,
            "particle_step": reduce("particle_step"), "multigrid_cg": reduce("multigrid_cg")}


def copy_calibration():
    import torch
    n = 256 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copied_bytes_per_dispatch": n * 8, "dispatches": 3}), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.profile_pass:
        profile_pass(json.loads(args.forms) if args.forms else None)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2506_09465_amd as P
    from synth import cavity_2d
    assert torch.cuda.is_available(), "needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.nongray_only:
        print(json.dumps(bench_nongray(P, dev, args.steps, 20, atomics_ceiling(P))), flush=True)
        return
    if args.c2_gray_only:
        print(json.dumps(bench_c2_gray(P, dev, args.steps, atomics_ceiling(P))), flush=True)
        return
    if args.persistent_only:
        print(json.dumps(bench_persistent(P, dev, args.steps, atomics_ceiling(P))), flush=True)
        return
    if args.expected_only:
        print(json.dumps(bench_expected(P, dev)), flush=True)
        return
    if args.batch_only:
        print(json.dumps(bench_batch(P, dev, args.batch)), flush=True)
        return

    # the four Kn problems are independent: each solver has a stream of its
    # own and every step is enqueued on all four before any is waited for, so
    # one problem's Newton CG (a few tens of workgroups) overlaps the others'
    # particle steps
    # (created longest particle step first: streams are spread over the
    # hardware queues in creation order, and the two long steps should not
    # share one)
    solvers = []
    for kn in sorted(KNS, reverse=True):
        w = cavity_2d(n=N_SIDE, kn=kn, particles=PARTICLES, newton=True, seed=0)
        solvers.append((kn, w, P.Solver(w, device=dev, tally_faces=P.FACES_EVERY,
                                        own_stream=True, cg_precond=P.PRECOND_MG)))
    solvers.sort(key=lambda t: t[0])

    def run_concurrent(n):
        # n iterations of every problem; each problem's next iteration is
        # enqueued as soon as its previous one is done
        rc = P.step_group([s for _, _, s in solvers], n)
        assert rc == 0, f"step failed with {rc}"

    # the particle-step form search of each problem (an untimed iteration, then
    # one per form: tiles of 256 and 512 threads, row stripes, row stripes in
    # pieces), one problem at a time so that each measurement has the GPU to
    # itself
    for _, _, s in solvers:
        assert s.step(5) == 0
    run_concurrent(args.warmup)
    # kernel pass: the same steps one problem at a time, for per-kernel times
    # (HIP events on each solver's stream) free of the other problems' kernels
    st0 = [s.stats() for _, _, s in solvers]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for _, _, s in solvers:
            rc = s.step(1)
            assert rc == 0, f"step failed with {rc}"
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = [s.stats() for _, _, s in solvers]
    seq_elapsed = t1 - t0
    # timed steps: the four problems concurrently
    fl0 = sum(s.stats()["tot_flights"] for _, _, s in solvers)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    run_concurrent(args.steps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    fl_timed = sum(s.stats()["tot_flights"] for _, _, s in solvers) - fl0

    elapsed = seq_elapsed
    K = args.steps
    # release the four solvers (and their streams' work) before anything else
    st_final = [s.stats() for _, _, s in solvers]
    tuning = {kn: s.march_tuning() for kn, _, s in solvers}
    for _, _, s in solvers:
        s.close()
    torch.cuda.synchronize()
    del st_final
    per_kn = {}
    tot = dict(flights=0, crossings=0, segments=0, ms_march=0.0, ms_cg=0.0, march_bytes=0,
               cg_bytes=0, cg_iters=0, launches=0)
    for (kn, w, s), a, b in zip(solvers, st0, st1):
        fl = b["tot_flights"] - a["tot_flights"]
        cr = b["tot_crossings"] - a["tot_crossings"]
        sg = b["tot_segments"] - a["tot_segments"]
        ms_m = b["ms_march"] - a["ms_march"]
        ms_c = b["ms_cg"] - a["ms_cg"]
        cgi = b["cg_iters_total"] - a["cg_iters_total"]
        mb = march_bytes(fl, cr, sg, b["n_emitters"] * K, False)
        cb = mgcg_bytes(cgi, w.nx, w.ny)
        per_kn[str(kn)] = {
            "flights_per_iter": fl // K, "crossings_per_flight": round(cr / max(fl, 1), 2),
            "ms_march": round(ms_m / K, 3), "ms_cg": round(ms_c / K, 3),
            "cg_iters": cgi // K, "flights_per_s_march": fl / (ms_m / 1e3) if ms_m else None,
            "crossings_per_s_march": cr / (ms_m / 1e3) if ms_m else None,
            "cg_us_per_iteration": round(ms_c * 1e3 / cgi, 3) if cgi else None,
            "march_GBs_algorithmic": mb / (ms_m / 1e3) / 1e9 if ms_m else None,
            "march_form": tuning[kn][0],
            "march_form_ms": {f: (round(v, 3) if v is not None else None)
                              for f, v in tuning[kn][1].items()},
        }
        for k, v in (("flights", fl), ("crossings", cr), ("segments", sg), ("ms_march", ms_m),
                     ("ms_cg", ms_c), ("march_bytes", mb), ("cg_bytes", cb), ("cg_iters", cgi)):
            tot[k] += v
        tot["launches"] += K

    src = source_hash()
    ceil = atomics_ceiling(P)
    counters = None if args.no_counters else collect_counters(
        {k: v["march_form"] for k, v in per_kn.items() if v.get("march_form")})
    cnt_ok = counters is not None and "error" not in counters
    n_l = tot["launches"]
    ps_ms = tot["ms_march"] / n_l
    cg_ms = tot["ms_cg"] / n_l
    # particle step: the algorithmic tally updates (one per face crossed and one
    # deposit or wall absorption per flight) against the LDS int64-atomic
    # ceiling, the best rate any placement of the tallies can reach
    tallies = (tot["crossings"] + tot["flights"]) / n_l
    ps_rate = tallies / (ps_ms / 1e3)
    ps = {"bound": "atomics", "achieved": ps_rate, "peak": ceil["lds_int64_per_s"],
          "unit": "tally atomics/s", "frac": round(ps_rate / ceil["lds_int64_per_s"], 5),
          "traffic": None, "avg_launch_ms": round(ps_ms, 4),
          "algorithmic_atomics_per_launch": int(tallies),
          "algorithmic_bytes_per_launch": int(tot["march_bytes"] / n_l),
          "share_of_sequential_step": round(tot["ms_march"] / (elapsed * 1e3), 3),
          "kernels": list(PS_KERNELS)}
    cg_b = tot["cg_bytes"] / n_l
    cg_rate = cg_b / (cg_ms / 1e3) / 1e9
    cg = {"bound": "hbm", "achieved": round(cg_rate, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
          "frac": round(cg_rate / HBM_PEAK_GBS, 5), "traffic": None,
          "avg_launch_ms": round(cg_ms, 4), "algorithmic_bytes_per_launch": int(cg_b),
          "us_per_cg_iteration": round(tot["ms_cg"] * 1e3 / max(tot["cg_iters"], 1), 3),
          "share_of_sequential_step": round(tot["ms_cg"] / (elapsed * 1e3), 3),
          "kernels": list(CG_KERNELS),
          "note": "latency-bound: group barriers and the fixed-order reductions of every "
                  "iteration, not bandwidth"}
    if cnt_ok:
        c = counters["particle_step"]
        sec = ps_ms / 1e3
        hb = c.get("hbm_bytes")
        ps["traffic"] = int(hb) if hb else None
        ps["measured"] = {
            "hbm": {"bytes_per_launch": hb, "achieved_GBs": hb / sec / 1e9 if hb else None,
                    "peak_GBs": HBM_PEAK_GBS,
                    "frac": round(hb / sec / 1e9 / HBM_PEAK_GBS, 5) if hb else None},
            "global_atomics": {"requests_per_launch": c["tcp_atomic_requests"],
                               "to_memory_per_launch": c["ea_atomic_requests"],
                               "achieved_per_s": c["tcp_atomic_requests"] / sec,
                               "peak_per_s": ceil["global_int64_2MB_per_s"],
                               "frac": round(c["tcp_atomic_requests"] / sec /
                                             ceil["global_int64_2MB_per_s"], 5),
                               "note": "atomic requests from the vector caches to L2 "
                                       "(TCP_TCC_ATOMIC_WITHOUT_RET_REQ) against int64 adds "
                                       "to random words, one request per lane"},
            "lds": {"wave_instructions_per_launch": c["lds_wave_instructions"],
                    "achieved_per_s": c["lds_wave_instructions"] / sec,
                    "peak_per_s": ceil["lds_int64_per_s"] / 64.0,
                    "frac": round(c["lds_wave_instructions"] / sec /
                                  (ceil["lds_int64_per_s"] / 64.0), 5),
                    "note": "every LDS instruction of the step (tally atomics, the tally "
                            "tiles' zeroing and flush, the pre-pass staging) against the "
                            "rate of full-wavefront LDS int64 atomics"},
            "occupancy": {"mean_waves_per_active_cu": c["mean_occupancy_waves_per_active_cu"],
                          "waves_per_launch": c["waves"]}}
        g = counters["multigrid_cg"]
        cg["traffic"] = int(g["hbm_bytes"]) if g.get("hbm_bytes") else None
        cg["measured"] = {"occupancy": {"mean_waves_per_active_cu":
                                        g["mean_occupancy_waves_per_active_cu"],
                                        "waves_per_launch": g["waves"]},
                          "lds_wave_instructions_per_launch": g["lds_wave_instructions"]}
    rooflines = {"particle_step": ps, "multigrid_cg": cg}
    dominant = "particle_step" if tot["ms_march"] >= tot["ms_cg"] else "multigrid_cg"
    roof = dict(rooflines[dominant])
    roof["kernel"] = dominant

    out = {
        "metric": "flights/s + time-to-steady (res<1e-6); batched vs sequential, same GPU",
        "value": fl_timed / (t3 - t2), "unit": "flights/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round((t3 - t2) / K * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+int64",
        "data": "synthetic",
        "config": {"workload": "2D gray square cavity 256x256, hot top wall, Kn in {0.01,0.1,1,10}, "
                               "1e7 particles/iteration, Newton (FP64 CG tol 1e-10, multigrid "
                               "V-cycle preconditioner), int64 "
                               "fixed-point tallies, face tallies every iteration; one step = one "
                               "iteration of each Kn (the four on their own streams, each "
                               "iteration enqueued as soon as the problem's previous one ends)",
                   "seed": 0, "parallelism": "single GPU"},
        "sequential": {"ms_per_step": round(seq_elapsed / K * 1e3, 3),
                       "flights_per_s": tot["flights"] / seq_elapsed,
                       "note": "the same steps one problem at a time; per_kn, roofline and "
                               "kernels come from this pass"},
        "per_kn": per_kn,
        "roofline": roof,
        "kernels": rooflines,
        "source_hash": src,
    }

    out["atomics_ceiling"] = ceil
    out["counters"] = counters

    if not args.no_tts:
        tts = {}
        for kn in KNS:
            w = cavity_2d(n=N_SIDE, kn=kn, particles=PARTICLES, newton=True, seed=0)
            s = P.Solver(w, device=dev, rng_mode=P.RNG_CRN, tally_faces=P.FACES_FINAL,
                         max_iters=100, res_tol=1e-6, cg_precond=P.PRECOND_MG)
            torch.cuda.synchronize()
            a = time.perf_counter()
            rc, T, qx, qy, st = s.solve()
            torch.cuda.synchronize()
            b = time.perf_counter()
            tts[str(kn)] = {"seconds": round(b - a, 4), "iterations": st["iters"], "rc": rc,
                            "final_res": st["res"], "cg_iters_total": st["cg_iters_total"]}
            s.close()
        out["time_to_steady"] = tts

    if args.batch:
        out["batched"] = bench_batch(P, dev, args.batch)

    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(P, dev)

    if not args.no_persistent:
        out["persistent"] = bench_persistent(P, dev, args.steps, ceil)

    if not args.no_expected:
        out["expected_value"] = bench_expected(P, dev)

    if not args.no_nongray:
        out["nongray"] = bench_nongray(P, dev, args.steps, 20, ceil)
        if not args.no_cpu_baseline:
            out["nongray"]["cpu_baseline"] = cpu_baseline_nongray()

    if not args.no_c0:
        out["c0_time_to_steady"] = bench_c0_time_to_steady(P, dev)

    if not args.no_c2_gray:
        out["c2_gray"] = bench_c2_gray(P, dev, 3, ceil)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
        host = host_cpu()
        out["cpu_baseline"]["host"] = host
        procs = max(1, min(16, host["usable_cores"] or 1))
        out["cpu_baseline"]["all_cores"] = cpu_baseline_all_cores(args.cpu_sample // 4, procs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
