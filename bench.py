#!/usr/bin/env python3
"""Frame-element gate updates per second on one MI355X.

Workload (default): the n=128 random Clifford+T circuits (2000 H/S/CNOT drawn
uniformly, 16 T at uniform slots, then 16 Z measurements), 1024 seeded
circuits per step (four tableau-track workgroups per compute unit: the track
of one circuit is one wavefront walking its gates in order, so a step of few
circuits leaves the device idle), run through the batched path (--path): one
batched reset and one sf_batch_run over all states per step, whose rounds
launch the tableau tracks of all frames together and their element kernels
together.  The same circuits three at a time (the smallest batch) and one at
a time (the plain path, on the leading circuits) are reported beside it.  U
counts, for every gate applied, the frame size just before it; value = U /
wall time of the timed steps, with states already resident in HBM.  The plain
path (one state at a time), the graph replay, the many-frame workloads, the
direct forms, the HBM probes, the Clifford-only circuits and the serving run
are reported beside it.

Prints one JSON line: metric, value, unit, the timing fields, the roofline of
the dominant kernel (achieved rate from HIP events around its launches in the
timed region, the peak it is held against, HBM traffic per launch from the
committed counter measurements when they match the current sources), the
oracle's rate on the host (cpu_baseline) and the extra workloads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz 32-bit ops; a 64-bit bitwise word op is two
PEAK_WORD_GOPS = 256 * 4 * 16 * 2.4 / 2
TERMINAL_OPS = None


def kernel_source_hash():
    """Hash of the device sources; HBM traffic figures measured with counters
    are reported only while the kernels are the ones they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("track.hip", "elem.hip", "sf_dev.h"):
        with open(os.path.join(ROOT, "paper_1712_03554_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary, or None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            tab = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = tab.get(kernel, {}).get(workload)
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def rec_stride(n):
    """Bytes of one per-gate record of the split tableau track: the rows (x
    and z words of n slots), the hull (31 vectors of W words) and its
    dimension, rounded to 256 bytes."""
    W = (n + 63) // 64
    b = n * 2 * W * 8 + 31 * W * 8 + 8
    return (b + 255) & ~255


def clifford_gate_count(circ, wl):
    """Device Clifford gates of a circuit (phase gates at multiples of pi/2
    other than the identity included)."""
    k = 0
    for op, q0, q1, q2, num, den in circ.gates:
        if op in (wl.H, wl.S, wl.SDG, wl.X, wl.Y, wl.Z, wl.CNOT, wl.CZ):
            k += 1
        elif op == wl.PHASE and (2 * num) % den == 0 and ((2 * num) // den) % 4 != 0:
            k += 1
    return k


def terminal_indices(circ, wl):
    """Indices of the gates that end a segment: non-Clifford phase gates and
    measurements (T, T-dagger, PHASE with an angle off the pi/2 grid, MEASURE)."""
    out = []
    for i, g in enumerate(circ.gates):
        op, num, den = g[0], g[4], g[5]
        if op in (wl.T, wl.TDG, wl.MEASURE):
            out.append(i)
        elif op == wl.PHASE and (2 * num) % den != 0:
            out.append(i)
        elif op in (wl.CPHASE, wl.TOF):
            raise ValueError("bench workloads use expanded gates only")
    return out


def accounting(state, circ, seed, wl, sizes=None, meas=None):
    """Untimed pass: U (sum over gates of |F| before the gate) and the hull
    dimension on entry to every segment launch (and, into sizes, |F| there;
    into meas, (d before, d after) of every measurement)."""
    state.reset(circ.init_bits, seed)
    terms = terminal_indices(circ, wl)
    U, K, d, pos = 0, 1, 0, 0
    seg_dims = []
    ends = terms + ([len(circ.gates) - 1] if (not terms or terms[-1] != len(circ.gates) - 1) else [])
    for t in ends:
        seg_dims.append(d)
        if sizes is not None:
            sizes.append(K)
        U += K * (t - pos + 1)
        k = state.step(t + 1 - pos)
        assert k == t + 1 - pos, (k, t, pos)
        K = state.frame_size()
        d_before, d = d, state.dim()
        if meas is not None and circ.gates[t][0] == wl.MEASURE:
            meas.append((d_before, d))
        pos = t + 1
    return U, seg_dims


def host_info():
    """Host core count and CPU model (from /proc/cpuinfo)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def _workload_circuit(kind, idx):
    from paper_1712_03554_amd import workloads as wl
    if kind == "steane":
        return wl.config3(idx), wl.derive_seed(3, idx)
    if kind == "uneven":
        return wl.config4(idx), wl.derive_seed(4, idx)
    if kind == "cfg2":
        return wl.config2(idx), wl.derive_seed(2, idx)
    if kind == "stab512":
        return wl.stabilizer_circuit(512, 9300 + 17 * 512 + idx % 4), idx
    return wl.config5_job(idx), wl.derive_seed(5, idx) ^ 0x5E


def _oracle_task(task):
    """One circuit on the oracle in a pool worker: (U, seconds)."""
    from oracle.frame import OracleFrame
    kind, idx = task
    c, seed = _workload_circuit(kind, idx)
    f = OracleFrame(c.n, c.init_bits, seed)
    t0 = time.perf_counter()
    sizes = f.run(c.array())
    return int(sizes.sum()), time.perf_counter() - t0


def _noop(_):
    return 0


def cpu_baseline(circ, seed):
    """The oracle on one full cfg2 circuit on one host thread (the headline
    comparison), plus the many-frame and served workloads with one circuit
    per task on a process pool over the host cores."""
    from oracle.frame import OracleFrame
    f = OracleFrame(circ.n, circ.init_bits, seed)
    arr = circ.array()
    t0 = time.perf_counter()
    sizes = f.run(arr)
    dt = time.perf_counter() - t0
    U = int(sizes.sum())
    host = host_info()
    out = {"value": U / dt, "unit": "frame-element gate updates/s", "cores": 1, "kind": "oracle",
           "sample": f"{circ.name}: one full circuit ({len(arr)} gates, U={U}) on one host thread, {dt:.2f} s",
           "host": host, "workloads": []}
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    from paper_1712_03554_amd import workloads as wl
    workers = max(1, min(16, host["nproc"] or 1))
    serve_idx = []
    for j in range(48):
        c = wl.config5_job(j)
        if not c.name.startswith("cfg5b"):
            serve_idx.append(j)
    legs = [("random Clifford+T, n=128 (the headline workload)", "cfg2", list(range(workers)),
             f"the first {workers} of its circuits, one per core"),
            ("Steane fault-injection trials", "steane", list(range(4096)), "all 4096 trials"),
            ("uneven random Clifford+T", "uneven", list(range(128)),
             "the first 128 of the 1024 circuits (n in 16..256)"),
            ("stabilizer circuits n=512 (beta = 1, then every qubit measured)", "stab512",
             list(range(workers)), f"{workers} circuits (4 distinct gate lists, one seed each), one per core"),
            ("served mix", "serve", serve_idx,
             f"the {len(serve_idx)} AQFT and uneven-shaped requests of the 48-request stream (the Cuccaro "
             "adders, 2^18..2^66 elements, take minutes to hours each on the oracle and are left out)")]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as pool:
        list(pool.map(_noop, range(4 * workers)))  # start every worker before timing
        for name, kind, idx, sample in legs:
            t0 = time.perf_counter()
            res = list(pool.map(_oracle_task, [(kind, i) for i in idx], chunksize=max(1, len(idx) // (8 * workers))))
            wall = time.perf_counter() - t0
            Us = sum(r[0] for r in res)
            out["workloads"].append({"workload": name, "value": Us / wall, "unit": "frame-element gate updates/s",
                                     "cores": workers, "kind": "oracle", "U": Us, "wall_s": wall,
                                     "cpu_s": sum(r[1] for r in res), "requests_per_s": len(idx) / wall,
                                     "sample": sample})
    return out


def clifford_only_wide(eng, wl, sizes=(512, 1024, 1500), frames=256, distinct=4, reps=2):
    """The Clifford-only workload on frames of more than 256 qubits (rows in
    device memory, one workgroup per frame): one circuit alone, and `frames`
    circuits (`distinct` gate lists, one seed per frame) in one batched run.
    U = gates applied (one element)."""
    import torch
    out = []
    for n in sizes:
        circs = [wl.stabilizer_circuit(n, 9300 + 17 * n + j) for j in range(distinct)]
        loaded = [eng.load(c.n, c) for c in circs]
        states = [loaded[j % distinct].state(circs[j % distinct].init_bits, j) for j in range(frames)]
        G = sum(len(circs[j % distinct]) for j in range(frames))
        st = states[0]
        st.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st.reset(circs[0].init_bits, 0)
            st.run()
        torch.cuda.synchronize()
        alone_s = (time.perf_counter() - t0) / reps

        def reset_all():
            for j, s in enumerate(states):
                s.reset(circs[j % distinct].init_bits, j)

        reset_all()
        eng.batch_run(states)
        torch.cuda.synchronize()
        tot = 0.0
        eng.profile(True, ["wide"])
        for _ in range(reps):
            reset_all()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eng.batch_run(states)
            torch.cuda.synchronize()
            tot += time.perf_counter() - t0
        kms, kn = eng.profile_read()["wide"]
        eng.profile(False)
        batch_s = tot / reps
        out.append({"workload": f"stabilizer circuits n={n}, {len(circs[0])} gates incl. {n} measurements",
                    "alone_ms_per_circuit": alone_s * 1e3, "alone_us_per_gate": alone_s / len(circs[0]) * 1e6,
                    "alone_gates_per_s": len(circs[0]) / alone_s, "batched_frames": frames,
                    "batched_ms": batch_s * 1e3, "batched_gates_per_s": G / batch_s,
                    "kernel_ms_per_launch": kms / max(1, kn),
                    "frame_sizes_after": sorted({s.frame_size() for s in states[:8]})})
        for s in states:
            s.close()
    return out


def batched_extra(eng, wl, name, circs, seeds, plain_sample):
    """Batched vs plain U/s on a many-frame workload: the batched form runs
    every frame of the workload per step; the plain form runs the first
    plain_sample frames one at a time (a rate, so the two compare)."""
    import torch
    loaded = [eng.load(c.n, c) for c in circs]
    states = [l.state(c.init_bits, s) for l, c, s in zip(loaded, circs, seeds)]
    Us = [accounting(st, c, s, wl)[0] for st, c, s in zip(states, circs, seeds)]

    def reset(idx):
        for i in idx:
            states[i].reset(circs[i].init_bits, seeds[i])

    import numpy as np
    import paper_1712_03554_amd as sf
    batch = sf.StateBatch(states)
    nmax = max(c.n for c in circs)
    bases = np.zeros((len(circs), nmax), dtype=np.uint8)
    for i, c in enumerate(circs):
        bases[i, :c.n] = np.asarray(c.init_bits, dtype=np.uint8)
    seed_arr = np.asarray(seeds, dtype=np.uint64)
    eng.batch_reset(batch, bases, seed_arr)
    eng.batch_run(batch)  # warm-up
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        eng.batch_reset(batch, bases, seed_arr)
        eng.batch_run(batch)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    g = eng.batch_graph(states, [c.init_bits for c in circs], seeds)
    g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.launch()
    torch.cuda.synchronize()
    tg = (time.perf_counter() - t0) / reps
    g.close()
    sub = range(min(plain_sample, len(states)))
    reset(sub)
    for i in sub:
        states[i].run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reset(sub)
    for i in sub:
        states[i].run()
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    for st in states:
        st.close()
    return {"workload": name, "frames": len(states), "U_per_step": int(sum(Us)),
            "graph_value": sum(Us) / tg, "graph_ms_per_step": tg * 1e3,
            "batched_value": sum(Us) / tb, "batched_ms_per_step": tb * 1e3,
            "plain_value": sum(Us[i] for i in sub) / tp, "plain_sample_frames": len(sub)}


def hbm_probe(eng, wl, d=26, det_gates=24, reps=3):
    """Element kernels in the HBM-bound regime: H then T on d qubits grows one
    frame to 2^d elements (d GROW segments), then det_gates T gates on those
    (now deterministic) qubits are phase-only passes over all 2^d slots
    (32 B per slot: read and write 16 B).  Their bandwidth is the difference
    of the segment-kernel time of the two circuits (with and without the
    passes) over the bytes of the passes."""
    import torch
    n = d + 4

    def circ(k):
        c = wl.Circuit(n, name=f"hbm-probe-d{d}-{k}")
        for q in range(d):
            c.h(q)
        for q in range(d):
            c.t(q)
        for i in range(k):
            c.t(i % d)
        return c

    seg_ms = []
    for k in (0, det_gates):
        c = circ(k)
        lc = eng.load(c.n, c)
        st = lc.state(c.init_bits, 3)
        st.run()
        torch.cuda.synchronize()
        eng.profile(True)
        for _ in range(reps):
            st.reset(c.init_bits, 3)
            st.run()
        torch.cuda.synchronize()
        prof = eng.profile_read()
        eng.profile(False)
        seg_ms.append(prof["segment"][0] / reps)
        K = st.frame_size()
        st.close()
    pass_bytes = 32.0 * (1 << d)
    ms = (seg_ms[1] - seg_ms[0]) / det_gates
    gbs = pass_bytes / (ms / 1e3) / 1e9
    return {"frame_elements": K, "slots": 1 << d, "bytes_per_pass": pass_bytes, "ms_per_pass": ms,
            "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
            "kernel": "sf_seg_kernel",
            "note": f"phase-only segment passes over 2^{d} complex128 slots ({(16 << d) >> 20} MiB per buffer)"}


def large_frame(eng, wl, m=12, reps=2):
    """Element kernels on a large frame of a real circuit: the Cuccaro adder
    of the served mix (m-bit registers, inputs in superposition, Toffolis as
    7-T networks) grows one frame to 2^(2m+2) elements.  Algorithmic bytes,
    a lower bound for every segment kind: each of the 2^d slots on entry is
    read once (16 B) and each of the |F| live elements written once (16 B); a
    split writes every slot of both halves, so it moves more than this."""
    import torch
    c = wl.cuccaro_adder(m, name=f"cuccaro-m{m}")
    lc = eng.load(c.n, c)
    st = lc.state(c.init_bits, 1)
    Ks = []
    U, dims = accounting(st, c, 1, wl, sizes=Ks)
    st.reset(c.init_bits, 1)
    st.run()
    torch.cuda.synchronize()
    eng.profile(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        st.reset(c.init_bits, 1)
        st.run()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    prof = eng.profile_read()
    eng.profile(False)
    seg_ms, seg_n = prof["segment"]
    seg_ms /= reps
    seg_bytes = sum(16.0 * (1 << d) + 16.0 * k for d, k in zip(dims, Ks))
    gbs = seg_bytes / (seg_ms / 1e3) / 1e9 if seg_ms > 0 else 0.0
    out = {"workload": f"Cuccaro adder m={m} ({c.n} qubits), inputs in superposition, 7-T Toffolis",
           "gates": len(c), "max_frame_log2": max(dims + [st.dim()]), "final_frame_size": st.frame_size(),
           "ms_per_circuit": wall * 1e3, "U": U, "value": U / wall,
           "segment_ms": seg_ms, "segment_launches": seg_n // reps,
           "track_ms": prof["track"][0] / reps,
           "element_roofline": {"bound": "hbm", "kernel": "sf_seg_kernel", "achieved": gbs,
                                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                                "bytes_per_circuit": seg_bytes,
                                "live_fraction": sum(Ks) / max(1.0, sum(float(1 << d) for d in dims)),
                                "bytes_per_live_element": seg_bytes / max(1, sum(Ks))}}
    st.close()
    return out


def clifford_only(eng, wl, sizes=(128, 256), batch=8, reps=3):
    """The paper's Clifford-only workload (random stabilizer circuits, n log2 n
    H/S/CNOT gates, then every qubit measured) at the sizes the library
    supports: one circuit at a time and `batch` circuits per batched run.  The
    frame keeps one element, so U = gates applied."""
    import torch
    out = []
    for n in sizes:
        circs = [wl.stabilizer_circuit(n, 9300 + 17 * n + j) for j in range(batch)]
        loaded = [eng.load(c.n, c) for c in circs]
        states = [l.state(c.init_bits, j) for j, (l, c) in enumerate(zip(loaded, circs))]
        st = states[0]
        st.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st.reset(circs[0].init_bits, 0)
            st.run()
        torch.cuda.synchronize()
        plain_s = (time.perf_counter() - t0) / reps
        bases = [c.init_bits for c in circs]
        seeds = list(range(batch))
        eng.batch_reset(states, bases, seeds)
        eng.batch_run(states)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            eng.batch_reset(states, bases, seeds)
            eng.batch_run(states)
        torch.cuda.synchronize()
        batch_s = (time.perf_counter() - t0) / reps
        sizes_after = [s.frame_size() for s in states]
        out.append({"workload": f"stabilizer circuits n={n}, {len(circs[0])} gates incl. {n} measurements",
                    "plain_ms_per_circuit": plain_s * 1e3, "plain_gates_per_s": len(circs[0]) / plain_s,
                    "batched_circuits": batch, "batched_ms": batch_s * 1e3,
                    "batched_gates_per_s": sum(len(c) for c in circs) / batch_s,
                    "frame_sizes_after": sorted(set(sizes_after))})
        for s in states:
            s.close()
    return out


def direct_vs_decomposed(eng, wl, reps=3):
    """Wall time per circuit (plain path, one frame) of the decomposed and the
    direct (double-cofactor) forms of controlled rotations and Toffolis."""
    import torch
    out = []
    for name, mk in (("AQFT n=18 (k<=6)", lambda d: wl.qft(18, [1, 0, 1] * 6, max_k=6, direct=d)),
                     ("Cuccaro adder m=10, inputs in superposition", lambda d: wl.cuccaro_adder(10, direct=d))):
        rec = {"workload": name}
        for direct in (False, True):
            c = mk(direct)
            lc = eng.load(c.n, c)
            st = lc.state(c.init_bits, 1)
            st.run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                st.reset(c.init_bits, 1)
                st.run()
            torch.cuda.synchronize()
            key = "direct" if direct else "decomposed"
            rec[key] = {"ms_per_circuit": (time.perf_counter() - t0) / reps * 1e3, "gates": len(c),
                        "frame_bound_log2": lc.info()[0], "final_frame_size": st.frame_size()}
            st.close()
        rec["speedup"] = rec["decomposed"]["ms_per_circuit"] / rec["direct"]["ms_per_circuit"]
        out.append(rec)
    return out


def serve_bench(eng, sf, wl, n_jobs, tick_segments, max_resident, budget_bytes, load_frac=0.7, direct=False):
    """Serving on the mixed request stream (AQFT 40%, Cuccaro adder 40%,
    random Clifford+T 20%).  First a saturation run (every job submitted at
    t=0) gives the batched capacity in jobs/s; then jobs arrive as a Poisson
    stream at load_frac of that capacity.  Latency = time from a job's arrival
    to its outcomes and frame size being on the host."""
    import numpy as np
    import torch
    jobs = [wl.config5_job(j, direct=direct) for j in range(n_jobs)]
    seeds = [wl.derive_seed(5, j) for j in range(n_jobs)]
    loaded, rejected_load = {}, 0
    tl0 = time.perf_counter()
    for j, c in enumerate(jobs):
        try:
            loaded[j] = eng.load(c.n, c)
        except sf.SFrameError as e:
            if e.status != sf.SF_E_TOO_LARGE:
                raise
            rejected_load += 1
    load_s = time.perf_counter() - tl0
    ok = sorted(loaded)
    print(f"serve: {len(ok)} of {n_jobs} jobs loadable ({load_s:.2f} s)", file=sys.stderr, flush=True)

    def run(arrivals):
        srv = sf.Server(eng, budget_bytes=budget_bytes, max_resident=max_resident, tick_segments=tick_segments)
        lat, rejected, pending, live = [], 0, list(range(len(ok))), {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while pending or live:
            now = time.perf_counter() - t0
            while pending and arrivals[pending[0]] <= now:
                i = pending.pop(0)
                j = ok[i]
                try:
                    live[srv.submit(loaded[j], jobs[j].init_bits, seeds[j])] = i
                except sf.SFrameError as e:
                    if e.status != sf.SF_E_TOO_LARGE:
                        raise
                    rejected += 1
            if not live:
                time.sleep(max(0.0, arrivals[pending[0]] - (time.perf_counter() - t0)))
                continue
            srv.tick()
            for jid, i in list(live.items()):
                stt, st = srv.poll(jid)
                if stt == srv.QUEUED or stt == srv.RESIDENT:
                    continue
                if stt != srv.DONE:
                    raise RuntimeError(f"served job {ok[i]} ended with status {stt}")
                st.outcomes()
                st.frame_size()
                lat.append(time.perf_counter() - t0 - arrivals[i])
                srv.release(jid)
                del live[jid]
        wall = time.perf_counter() - t0
        ticks = srv.stats()["ticks"]
        srv.close()
        return np.array(lat), wall, rejected, ticks

    lat_sat, wall_sat, rej_sat, ticks_sat = run([0.0] * len(ok))
    capacity = len(lat_sat) / wall_sat
    lam = load_frac * capacity
    rng = np.random.default_rng(wl.derive_seed(5, 1 << 20))
    arrivals = np.cumsum(rng.exponential(1.0 / lam, size=len(ok))).tolist()
    lat, wall, rej, ticks = run(arrivals)
    return {"jobs": n_jobs, "served": int(len(lat)), "rejected_too_large": rejected_load + rej,
            "capacity_jobs_per_s": capacity, "lambda_jobs_per_s": lam, "offered_load": load_frac,
            "throughput_jobs_per_s": len(lat) / wall, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "max_ms": float(lat.max() * 1e3),
            "saturated_p50_ms": float(np.percentile(lat_sat, 50) * 1e3), "ticks": ticks,
            "tick_segments": tick_segments, "max_resident": max_resident, "budget_bytes": budget_bytes,
            "circuit_load_ms_mean": load_s / n_jobs * 1e3}


def calib_copy(mib):
    """One device-to-device copy of mib MiB: the reference for the HBM byte
    counters (its FETCH_SIZE / WRITE_SIZE should read mib MiB each)."""
    if mib <= 0:
        return
    import torch
    src = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--jobs", type=int, default=1024,
                    help="circuits per step (1024: four tableau-track workgroups per compute unit)")
    ap.add_argument("--plain-jobs", type=int, default=3,
                    help="leading circuits the plain form runs one at a time (a rate)")
    ap.add_argument("--workload", default="cfg2", choices=["cfg2", "cfg2L"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--path", default="batched", choices=["graph", "batched", "plain"])
    ap.add_argument("--serve-jobs", type=int, default=48, help="0 skips the serving run")
    ap.add_argument("--no-extra", action="store_true", help="skip the many-frame batched workloads")
    ap.add_argument("--probe-only", action="store_true",
                    help="run only the HBM-bound element probe and print its JSON (for counter runs)")
    ap.add_argument("--large-only", action="store_true",
                    help="run only the large-frame circuit (element kernels on a 2^26-element frame)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, one device-to-device copy of this size (counter calibration)")
    ap.add_argument("--tune-lo", type=int, default=8)
    ap.add_argument("--tune-hi", type=int, default=26, help="below --tune-lo: no autotuning")
    ap.add_argument("--tick-segments", type=int, default=8)
    ap.add_argument("--max-resident", type=int, default=32)
    ap.add_argument("--serve-budget-gib", type=float, default=128.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1712_03554_amd as sf
    from paper_1712_03554_amd import workloads as wl

    eng = sf.Engine(0)
    tuned = eng.autotune(args.tune_lo, args.tune_hi) if args.tune_hi >= args.tune_lo else {}
    if args.probe_only:
        probe = hbm_probe(eng, wl)
        calib_copy(args.calib_copy_mib)
        print(json.dumps({"element_hbm_probe": probe}), flush=True)
        return
    if args.large_only:
        rec = large_frame(eng, wl)
        calib_copy(args.calib_copy_mib)
        print(json.dumps({"large_frame": rec}), flush=True)
        return
    if args.workload == "cfg2":
        circs = [wl.config2(j) for j in range(args.jobs)]
        seeds = [wl.derive_seed(2, j) for j in range(args.jobs)]
        wname = "random Clifford+T, n=128, 2000 H/S/CNOT + 16 T, measure 16 qubits"
    else:
        circs = [wl.config2(j, n_t=24) for j in range(args.jobs)]
        seeds = [wl.derive_seed(22, j) for j in range(args.jobs)]
        wname = "random Clifford+T, n=128, 2000 H/S/CNOT + 24 T, measure 16 qubits (HBM probe)"
    loaded = [eng.load(c.n, c) for c in circs]
    states = [l.state(c.init_bits, s) for l, c, s in zip(loaded, circs, seeds)]
    bounds = [l.info()[0] for l in loaded]

    U_each, seg_dims, seg_sizes, meas_dims = [], [], [], []
    for st, c, s in zip(states, circs, seeds):
        Ks, Ms = [], []
        U, dims = accounting(st, c, s, wl, sizes=Ks, meas=Ms)
        meas_dims.append(Ms)
        U_each.append(U)
        seg_dims.append(dims)
        seg_sizes.append(Ks)
    U_total = sum(U_each)
    n_plain = max(1, min(args.plain_jobs, len(states)))
    U_plain = sum(U_each[:n_plain])
    n_small = min(3, len(states))
    U_small = sum(U_each[:n_small])

    def plain_step():
        for st, c, s in list(zip(states, circs, seeds))[:n_plain]:
            st.reset(c.init_bits, s)
            st.run()

    bases = [c.init_bits for c in circs]
    # the batched resets take the basis bits packed once (host-side input
    # format), the seeds as a uint64 array; each step still uploads both and
    # initialises every state on the device
    words = sf.pack_bases(bases)
    seed_arr = np.asarray([int(x) & ((1 << 64) - 1) for x in seeds], dtype=np.uint64)

    batch = sf.StateBatch(states)

    def batched_step():
        eng.batch_reset(batch, words, seed_arr)
        eng.batch_run(batch)

    small = sf.StateBatch(states[:n_small])
    words_small = sf.pack_bases(bases[:n_small])

    def small_step():
        eng.batch_reset(small, words_small, seed_arr[:n_small])
        eng.batch_run(small)

    graph = None

    def graph_step():
        graph.launch()

    def timed(fn, U):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / args.steps
        return U / dt, dt * 1e3

    # the other forms, timed for the record
    plain_value, plain_ms = timed(plain_step, U_plain)
    small_value, small_ms = timed(small_step, U_small)
    batched_value, batched_ms = timed(batched_step, U_total)
    graph = eng.batch_graph(states, [c.init_bits for c in circs], seeds)
    graph_value, graph_ms = timed(graph_step, U_total)

    one_step = {"graph": graph_step, "batched": batched_step, "plain": plain_step}[args.path]
    U_one = U_plain if args.path == "plain" else U_total
    step_circs = circs[:n_plain] if args.path == "plain" else circs
    # untimed pass with every kernel kind timed: the breakdown per kind
    eng.profile(True)
    for _ in range(args.steps):
        one_step()
    torch.cuda.synchronize()
    prof_all = eng.profile_read()
    eng.profile(False)
    kinds = {k: v for k, v in prof_all.items() if v[1] > 0}
    # the dominant kernel on the step's critical path: when the batched
    # forms overlap rounds (circuits with a range cut every 1024 gates), the
    # phase kernel of a round runs beside the next round's tracks, so the
    # chain of tracks is on the critical path and the phase launches only
    # partly; their summed time then overstates their share
    overlapped = args.path != "plain" and any(len(c.gates) > 1024 for c in step_circs)
    crit = {k: v for k, v in kinds.items() if not (overlapped and k == "phase")}
    dom = max(crit, key=lambda k: crit[k][0])
    # timed region: HIP events around the dominant kernel's launches only
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    eng.profile(True, kinds=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = eng.profile_read()
    eng.profile(False)
    cyc = {}
    for st in states:
        for k, v in st.track_cycles().items():
            cyc[k] = cyc.get(k, 0) + v
    elapsed = t1 - t0
    value = args.steps * U_one / elapsed

    # roofline of the dominant kernel (its launches timed in the timed region)
    seg_bytes_per_step = sum(32.0 * (1 << d) for dims in seg_dims for d in dims)
    # how full the hulls are: elements on entry to the segment launches over
    # the slots those launches stream
    live_elems = sum(k for ks in seg_sizes for k in ks)
    live_frac = live_elems / max(1.0, sum(float(1 << d) for dims in seg_dims for d in dims))
    seg_ms, seg_n = (prof if dom == "segment" else prof_all)["segment"]
    seg_ach = (seg_bytes_per_step * args.steps / max(seg_n, 1)) / (seg_ms / 1e3 / max(seg_n, 1)) / 1e9 \
        if seg_n else 0.0
    elem_roof = {"bound": "hbm", "kernel": "sf_seg_kernel" if args.path == "plain" else "sf_seg_batch",
                 "achieved": seg_ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": seg_ach / PEAK_HBM_GBS,
                 "traffic": measured_traffic("sf_seg_kernel" if args.path == "plain" else "sf_seg_batch",
                                             args.workload),
                 "live_fraction": live_frac, "bytes_per_live_element": seg_bytes_per_step / max(1, live_elems),
                 "note": "32 B per slot (read + write of 16 B) over 2^d slots per segment launch; "
                         "live_fraction = frame elements / hull slots over those launches"}
    def kind_ms(kind):
        """(ms, launches) of a kernel kind: from the timed region for the
        dominant kind, else from the untimed pass over the same steps."""
        return (prof if dom == kind else prof_all).get(kind, (0.0, 0))

    wset = sorted({(c.n + 63) // 64 for c in circs})
    # tableau track: one pass over the n rows per gate (4 n W 64-bit words)
    tr_ms, tr_n = kind_ms("track")
    words_per_step = sum(len(c.gates) * 4 * c.n * ((c.n + 63) // 64) for c in step_circs)
    ach = (words_per_step * args.steps / tr_n) / (tr_ms / 1e3 / tr_n) / 1e9 if tr_n else 0.0
    kname = ("sf_track_one<%d>" if args.path == "plain" else "sf_track_many<%d>") % wset[-1]
    track_roof = {"bound": "alu", "kernel": kname, "avg_launch_us": tr_ms / tr_n * 1e3 if tr_n else None,
                  "achieved": ach, "peak": PEAK_WORD_GOPS,
                  "unit": "G 64-bit word-ops/s", "frac": ach / PEAK_WORD_GOPS,
                  "traffic": measured_traffic(kname, args.workload),
                  "note": "one wavefront per circuit walks the gates; bound by the dependent LDS/VALU latency "
                          "of that wavefront, not by throughput"}
    # phase kernel: reads one record (the state after the gate) per Clifford
    # gate of a frame in split form (n <= 128)
    ph_ms, ph_n = kind_ms("phase")
    ph_bytes = sum(clifford_gate_count(c, wl) * rec_stride(c.n) for c in step_circs if c.n <= 128)
    ph_ach = (ph_bytes * args.steps / ph_n) / (ph_ms / 1e3 / ph_n) / 1e9 if ph_n else 0.0
    pname = ("sf_phase_one<%d>" if args.path == "plain" else "sf_phase_many<%d>") % min(2, wset[-1])
    phase_roof = {"bound": "hbm", "kernel": pname, "avg_launch_us": ph_ms / ph_n * 1e3 if ph_n else None,
                  "achieved": ph_ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ph_ach / PEAK_HBM_GBS,
                  "traffic": measured_traffic(pname, args.workload),
                  "note": "one record (rows and hull after the gate) read per Clifford gate; runs beside the "
                          "next round's tracks, so its launches share the SIMDs with them"}
    # measurements: the reduction reads the 2^d slots before (16 B each); the
    # filter reads the kept 2^d' slots and writes them (32 B each)
    step_meas = meas_dims[:n_plain] if args.path == "plain" else meas_dims
    red_bytes = sum(16.0 * (1 << a) for ms in step_meas for a, _ in ms)
    fil_bytes = sum(32.0 * (1 << b) for ms in step_meas for _, b in ms)

    def hbm_roof(kind, kname, nbytes, note):
        ms_, n_ = kind_ms(kind)
        a = (nbytes * args.steps / n_) / (ms_ / 1e3 / n_) / 1e9 if n_ else 0.0
        return {"bound": "hbm", "kernel": kname, "avg_launch_us": ms_ / n_ * 1e3 if n_ else None,
                "achieved": a, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": a / PEAK_HBM_GBS,
                "traffic": measured_traffic(kname, args.workload), "bytes_per_step": nbytes, "note": note}

    batched_names = args.path != "plain"
    meas_roof = {
        "reduce": hbm_roof("meas_reduce", "sf_meas_reduce_batch" if batched_names else "sf_meas_reduce",
                           red_bytes, "16 B read per hull slot before the measurement"),
        "filter": hbm_roof("meas_filter", "sf_meas_apply_batch" if batched_names else "sf_meas_filter",
                           fil_bytes, "32 B (read + write) per kept slot; launches of many blocks draw the coin "
                                      "in a kernel of their own and filter with sf_meas_apply_batch, the others "
                                      "with sf_meas_filter_batch, whose blocks also sum the reduction partials"),
    }
    roof = dict({"segment": elem_roof, "phase": phase_roof, "meas_reduce": meas_roof["reduce"],
                 "meas_filter": meas_roof["filter"]}.get(dom, track_roof))
    line = {
        "metric": "frame-element gate updates/s",
        "value": value,
        "unit": "frame-element gate updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": wname, "circuits_per_step": len(step_circs), "path": args.path,
                   "rounds_overlapped": overlapped,
                   "U_per_step": U_one, "frame_bound_log2_max": max(bounds),
                   "seeds": "splitmix64 stream of master seed 20171210, config 2, circuits 0..%d" % (len(circs) - 1)},
        "plain_value": plain_value,
        "plain_ms_per_step": plain_ms,
        "plain_circuits": n_plain,
        "batched_value": batched_value,
        "batched_ms_per_step": batched_ms,
        "graph_value": graph_value,
        "graph_ms_per_step": graph_ms,
        "three_circuit_batched_value": small_value,
        "three_circuit_batched_ms_per_step": small_ms,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kinds.items()},
        "kernel_launches_per_step": {k: v[1] / args.steps for k, v in kinds.items()},
        "roofline": roof,
        "track_roofline": track_roof,
        "phase_roofline": phase_roof,
        "element_roofline": elem_roof,
        "measurement_rooflines": meas_roof,
        "track_cycles_last_step": cyc,
        "autotune": {str(d): {"block": b, "grid": g, "ms": round(t, 4)} for d, (b, g, t) in tuned.items()},
    }
    if not args.no_extra:
        c3 = [wl.config3(t) for t in range(4096)]
        c4 = [wl.config4(j) for j in range(1024)]
        line["batched_workloads"] = [
            batched_extra(eng, wl, "Steane fault-injection trials, 4096 x 13 qubits", c3,
                          [wl.derive_seed(3, t) for t in range(4096)], 256),
            batched_extra(eng, wl, "uneven random Clifford+T, 1024 circuits, n in 16..256", c4,
                          [wl.derive_seed(4, j) for j in range(1024)], 16),
            # the large-frame variant of the headline workload: 24 T gates,
            # frames of up to 2^21 elements (64 circuits per step)
            batched_extra(eng, wl, "random Clifford+T, n=128, 2000 H/S/CNOT + 24 T, measure 16 qubits, "
                          "64 circuits", [wl.config2(j, n_t=24) for j in range(64)],
                          [wl.derive_seed(22, j) for j in range(64)], 2),
        ]
    if not args.no_extra:
        line["direct_forms"] = direct_vs_decomposed(eng, wl)
        line["element_hbm_probe"] = hbm_probe(eng, wl)
        line["large_frame"] = large_frame(eng, wl)
        line["clifford_only"] = clifford_only(eng, wl) + clifford_only_wide(eng, wl)
    if args.serve_jobs > 0:
        line["serve"] = serve_bench(eng, sf, wl, args.serve_jobs, args.tick_segments, args.max_resident,
                                    int(args.serve_budget_gib * (1 << 30)))
        line["serve_direct_forms"] = serve_bench(eng, sf, wl, args.serve_jobs, args.tick_segments,
                                                 args.max_resident, int(args.serve_budget_gib * (1 << 30)),
                                                 direct=True)
    if not args.no_cpu and args.workload == "cfg2":
        line["cpu_baseline"] = cpu_baseline(circs[0], seeds[0])
    calib_copy(args.calib_copy_mib)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
