#!/usr/bin/env python3
"""Benchmark: gate HBM bandwidth of the MI355X state-vector simulator.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 30] [--dtype c128]

One step is the per-gate workload at n = 30 complex128 (16 GiB state):
H and one Haar-random U on every target qubit 0..n-1, a controlled-U on 64
random (control, target) pairs, a 1000-gate random circuit (1q / controlled-U
mix, run through the circuit executor) and the per-qubit probabilities.
Inputs are synthetic and seeded; the state stays resident in HBM.

`value` = algorithmic HBM bytes of the step / step time: the paper's
per-gate byte counts (qHiPSTER Table 2: 2 * 2^n * b for a single-qubit gate,
2^n * b for a controlled gate with both qubits local) for the per-gate sweep,
2 * 2^n * b per pass of the fused circuit (as planned by qs_plan) and
2^n * b for the probability pass (b = bytes per amplitude).  The circuit's
"effective" bandwidth in the paper's sense (per-gate bytes of all its gates
/ time, Sec. 5.4) is reported separately and may exceed the HBM peak.

Extra objects on the same JSON line: `roofline` for the dominant kernel
(timed with HIP events on the stream the kernels run on), `cpu_baseline`
(the CPU oracle on a bounded sample), `stream_copy` (measured B_mem) and
per-category detail.  Further sections (each skippable): n=33 / n=34 large
states, the QFT / IQFT fused-vs-unfused sweep (n = 18..31, effective
bandwidth in the paper's sense), dense k-qubit gates (k = 1..5), adjoint vs
parameter-shift gradients
(n=20, n=28), and the batched persistent launch (4096 small ansatz
circuits, energy + gradient).  One GPU only: --gpus above 1 exits with a
message.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0  # MI355X HBM3E, AMD published peak
# Compiled fused passes time each of their tile orders (eight at the sizes
# timed here) on one launch apiece before keeping the fastest: this many
# untimed calls precede every timed fused run.
TUNE_CALLS = 8


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--dtype", choices=["c128", "c64"], default="c128")
    ap.add_argument("--ncu", type=int, default=64)
    ap.add_argument("--circuit-gates", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the n=33/34 (128 GiB) section")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint vs parameter-shift section")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-launch section")
    ap.add_argument("--no-qft", action="store_true",
                    help="skip the QFT/IQFT fused-vs-unfused sweep (n = 18..31)")
    ap.add_argument("--no-kq", action="store_true", help="skip the dense k-qubit gate section")
    ap.add_argument("--no-reorder", action="store_true", help="skip the qubit-reordering section")
    ap.add_argument("--ps-pairs", type=int, default=8,
                    help="parameter-shift pairs timed at n=28 (extrapolated to all 2P sweeps)")
    ap.add_argument("--cpu-n", type=int, default=0, help="qubits of the CPU-oracle sample (0 = auto)")
    ap.add_argument("--workload-only", choices=["circuit", "qft", "iqft", "adjoint", "batch", "cu-line", "gates"],
                    help="run one workload once after a warmup, plus a 4 GiB STREAM copy, and exit "
                         "(for hardware-counter runs): the 1000-gate random circuit, the QFT or IQFT on "
                         "all qubits at --n/--dtype, the n = 28 ansatz energy + gradient (--dtype), "
                         "the 4096-circuit batch (--dtype), or controlled gates with control qubits "
                         "0..3 and target 20 at --n/--dtype (twice each; QS_CU_COMPACT_FROM picks the "
                         "enumeration), or the main step's streamed gates at --n/--dtype (H and a Haar U "
                         "on every target, then the controlled-U pairs)")
    return ap.parse_args()


def workload_only(args) -> None:
    """One workload, once, after an untimed warmup (which compiles the pass
    kernels), then the STREAM copy used to calibrate the traffic counters."""
    import numpy as np
    import torch

    import circuits as C
    import paper_1601_07195_amd.qs as Q

    torch.cuda.set_device(0)
    dtype = Q.QS_C128 if args.dtype == "c128" else Q.QS_C64
    w = args.workload_only
    if w in ("circuit", "qft", "iqft"):
        n = args.n
        ops = {"circuit": lambda: C.random_circuit(n, args.circuit_gates, np.random.default_rng(C.SEED_BASE + 1)),
               "qft": lambda: C.qft_circuit(n), "iqft": lambda: C.iqft_circuit(n)}[w]().ops
        st = Q.State(n, dtype)
        # untimed runs: kernels compiled, then every tile order timed
        for _ in range(TUNE_CALLS):
            st.run(ops)
            torch.cuda.synchronize()
        log(f"[bench] {w} n={n} {args.dtype}: warmup done")
        st.run(ops)
        torch.cuda.synchronize()
        del st
    elif w == "gates":
        n = args.n
        u, pairs = C.workload_sweep(n, args.ncu, C.SEED_BASE + 1)
        st = Q.State(n, dtype)
        for k in range(n):
            st.apply_1q(k, C.H_GATE)
            st.apply_1q(k, u)
        for c, t in pairs:
            st.apply_cu(c, t, u)
        torch.cuda.synchronize()
        del st
    elif w == "cu-line":
        n = args.n
        st = Q.State(n, dtype)
        u = C.haar_unitary(np.random.default_rng(C.SEED_BASE + 9))
        for c in range(4):
            for _ in range(2):
                st.apply_cu(c, 20, u)
        torch.cuda.synchronize()
        del st
    elif w == "adjoint":
        n = 28
        circ, ham = C.workload_ansatz(n, 20, 100)
        st = Q.State(n, dtype)
        lam = Q.State(n, dtype, init=False)
        for _ in range(TUNE_CALLS + 1):
            st.init_basis(0)
            Q.grad_adjoint(st, lam, circ.ops, circ.theta, ham.codes, ham.coeff)
            torch.cuda.synchronize()
        del st, lam
    else:
        wl = C.workload_batch(4096)
        b = Q.Batch([(c.n, c.ops, c.theta, h.codes, h.coeff) for c, h in wl], dtype)
        b.run_flat()
        b.run_flat()
        torch.cuda.synchronize()
        b.close()
    torch.cuda.empty_cache()
    cs = 4 << 30
    src = torch.empty(cs // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    Q.qs_stream_copy(src, dst)
    torch.cuda.synchronize()
    log(f"[bench] workload {w} done")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


class EventTimer:
    """HIP events (torch.cuda.Event) recorded on the stream the library
    launches on; durations are read after the timed region."""

    def __init__(self, stream):
        self.stream = stream
        self.pending = {}

    def measure(self, key, fn):
        import torch
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        fn()
        e1.record(self.stream)
        self.pending.setdefault(key, []).append((e0, e1))

    def collect(self):
        out = {}
        for k, lst in self.pending.items():
            out[k] = [a.elapsed_time(b) * 1e-3 for a, b in lst]
        self.pending = {}
        return out


def measured_traffic(kernel: str, workload: str, key: str = ""):
    """HBM bytes per launch of `kernel` on `workload` from the rocprofv3 PMC
    summary committed under profiles/ (FETCH_SIZE and WRITE_SIZE, scaled by
    the same counters on the STREAM-copy kernel), or None when there is no
    such summary or the kernel's source has changed since it was taken.  A
    summary of several workloads holds one `traffic_bytes_per_launch.<key>`
    line per workload."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    want = "traffic_bytes_per_launch" + (f".{key}" if key else "")
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith(("traffic_bytes_per_launch", "source_file", "source_sha256")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    try:
        h = hashlib.sha256()
        for f in fields["source_file"].split(","):
            h.update(open(os.path.join(ROOT, f.strip()), "rb").read())
        if h.hexdigest() != fields["source_sha256"]:
            return None
        return float(fields[want])
    except (KeyError, OSError, ValueError):
        return None


# LDS peak for the batch kernel's roofline: 128 bytes per clock per CU
# (one 128-byte LDS access per clock), 256 CUs at 2.4 GHz.
PEAK_LDS_GBPS = 128 * 256 * 2.4


def section_rooflines(line):
    """Rooflines of the kernels the sections after the main step time: the
    QFT / IQFT passes (phase runs) at n = 30 complex128 and n = 31 complex64,
    the adjoint's forward and reverse passes at n = 28, and the batch kernel
    (LDS-bound: its modelled LDS bytes against the LDS peak)."""
    out = {}

    def put(name, launches, nbytes, ms, traffic, bound="hbm", peak=PEAK_HBM_GBPS):
        gbps = nbytes / (ms * 1e-3) / 1e9
        out[name] = {"bound": bound, "launches_per_step": launches, "bytes_per_launch": nbytes,
                     "mean_launch_ms": round(ms, 4), "achieved_GBps": round(gbps, 1), "peak_GBps": round(peak, 1),
                     "frac": round(gbps / peak, 4), "traffic": traffic}

    q = line.get("qft_fused_vs_unfused") or {}
    for dt, n, b in (("c128", 30, 16), ("c64", 31, 8)):
        rows = q.get(dt, {}).get(str(n))
        if not rows:
            continue
        for kind in ("qft", "iqft"):
            r = rows[kind]
            put(f"qs_pass_* ({kind.upper()} phase runs, n={n} {dt})", r["passes_fused"], 2 * (1 << n) * b,
                r["fused_s"] / r["passes_fused"] * 1e3,
                measured_traffic("qs_pass_compiled_phase_runs", "qft_iqft", f"{kind}_{dt}_n{n}"))
    adj = (line.get("adjoint_vs_param_shift") or {}).get("n28", {}).get("sweeps", {})
    for dt, b in (("c128", 16), ("c64", 8)):
        sw = adj.get(dt)
        if not sw:
            continue
        S = (1 << 28) * b
        put(f"qs_pass_* (adjoint forward sweep, n=28 {dt})", sw["forward_passes"], 2 * S, sw["forward_pass_ms"],
            measured_traffic("qs_pass_compiled_adjoint", "n28", f"forward_{dt}"))
        put(f"qs_pass_* (adjoint reverse sweep, n=28 {dt})", sw["reverse_passes"], 4 * S, sw["reverse_pass_ms"],
            measured_traffic("qs_pass_compiled_adjoint", "n28", f"reverse_{dt}"))
    bt = (line.get("batch") or {}).get("c128")
    if bt:
        put("k_batch (4096 circuits, c128)", 1, bt["lds_bytes_model"], bt["batch_s"] * 1e3, None,
            bound="lds", peak=PEAK_LDS_GBPS)
    return out


def cpu_baseline(n_gpu: int, u, pairs, args):
    """The CPU oracle, as it stands, on a bounded sample of the same
    per-gate workload: H and U on every target and eight controlled-U gates
    on the host's threads (at most 16), then H on the lowest and highest
    target on one thread."""
    import numpy as np

    import circuits as C
    import oracle as O

    threads = min(16, os.cpu_count() or 1)
    n = args.cpu_n
    if n <= 0:
        n = n_gpu
        try:
            import psutil
            avail = psutil.virtual_memory().available
            while n > 20 and (1 << n) * 16 * 2.5 > avail:
                n -= 1
        except Exception:
            n = min(n, 26)
    psi = O.basis_state(n)
    gates = []
    for k in range(n):
        gates.append(("1q", k, C.H_GATE))
        gates.append(("1q", k, u))
    for c, t in pairs[:8]:
        gates.append(("cu", (c % n, t % n) if c % n != t % n else (0, n - 1), u))
    S = (1 << n) * 16

    def run(gs):
        nbytes = 0
        t0 = time.perf_counter()
        for kind, q, m in gs:
            if kind == "1q":
                O.apply_1q(psi, n, q, m)
                nbytes += 2 * S
            else:
                O.apply_cu(psi, n, q[0], q[1], m)
                nbytes += S
        return nbytes, time.perf_counter() - t0

    O.set_threads(threads)
    nbytes, dt = run(gates)
    O.set_threads(1)
    nb1, dt1 = run([("1q", 0, C.H_GATE), ("1q", n - 1, C.H_GATE)])
    del psi
    out = {
        "value": round(nbytes / dt / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
        "sample": f"complex128 n={n}: H and Haar U on all {n} targets + {len(gates) - 2 * n} "
                  f"controlled-U, {len(gates)} gates, {dt:.2f} s",
        "one_core_GBps": round(nb1 / dt1 / 1e9, 3),
        "one_core_sample": f"H on targets 0 and {n - 1}, {dt1:.2f} s",
    }
    out.update(host_info(threads))
    out["host_stream_copy_GBps"] = host_stream_copy(np, threads)
    out["oracle_vs_host_copy"] = round(out["value"] / out["host_stream_copy_GBps"], 3)
    out["workloads"] = oracle_workloads(np, C, O, threads)
    return out


def host_info(threads: int) -> dict:
    """The host the oracle ran on: logical CPUs, the CPU model, and the share
    used (the GPU machine grants 16 threads per GPU whatever the CPU count)."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "threads_used": threads,
            "threads_note": "oracle threads capped at the 16-thread CPU share of one GPU"}


def host_stream_copy(np, threads: int) -> float:
    """Host STREAM-copy bandwidth (the paper's B_mem definition, Sec. 5.2):
    a 4 GiB float64 copy split over the oracle's threads (numpy releases the
    GIL while copying), best of three, counted as read + write bytes."""
    import concurrent.futures as cf
    a = np.ones((1 << 29,), dtype=np.float64)
    b = np.empty_like(a)
    parts = np.array_split(np.arange(a.size), threads)
    spans = [(int(p[0]), int(p[-1]) + 1) for p in parts if p.size]
    best = 0.0
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda r: np.copyto(b[r[0]:r[1]], a[r[0]:r[1]]), spans))
        for _ in range(3):
            t0 = time.perf_counter()
            list(ex.map(lambda r: np.copyto(b[r[0]:r[1]], a[r[0]:r[1]]), spans))
            best = max(best, 2 * a.nbytes / (time.perf_counter() - t0) / 1e9)
    del a, b
    return round(best, 2)


def oracle_workloads(np, C, O, threads: int) -> dict:
    """The oracle on the small workloads in full: the 200-gate n = 20 circuit
    with its probabilities, and the n = 20 ansatz energy; at n = 28 the
    ansatz's parameter shift extrapolated from ten timed gates (labelled)."""
    out = {}
    O.set_threads(threads)
    circ = C.workload_gates(20, 200)
    t0 = time.perf_counter()
    psi = O.run(circ.ops, 20)
    O.probabilities(psi, 20)
    out["n20_200_gates_and_probabilities_s"] = round(time.perf_counter() - t0, 3)
    ac, ham = C.workload_ansatz(20, 20, 100)
    t0 = time.perf_counter()
    O.energy(ac.ops, 20, ac.theta, ham.codes, ham.coeff)
    t_e20 = time.perf_counter() - t0
    out["n20_ansatz_energy_s"] = round(t_e20, 3)
    out["n20_ansatz_param_shift_s_extrapolated"] = round(2 * ac.nparams * t_e20, 1)
    a28, h28 = C.workload_ansatz(28, 20, 100)
    psi = O.basis_state(28)
    t0 = time.perf_counter()
    O.run(a28.ops[:10], 28, a28.theta, psi=psi)
    per_gate = (time.perf_counter() - t0) / 10
    t_e28 = per_gate * len(a28.ops)
    out["n28_ansatz_energy_s_extrapolated"] = round(t_e28, 1)
    out["n28_ansatz_param_shift_s_extrapolated"] = round(2 * a28.nparams * t_e28, 0)
    out["note"] = "extrapolated entries: time of 10 gates (n = 28) or one energy (n = 20) times the gate or sweep count"
    del psi
    return out


def timed(fn, stream, reps=1, warm=1):
    """Mean seconds of fn() over reps, with HIP events on `stream` after
    `warm` untimed calls (TUNE_CALLS for fused runs, so that the timed calls
    run each compiled pass in its chosen tile order)."""
    import torch
    for _ in range(warm):
        fn()
        torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def large_section(Q, C, np, torch):
    """The 128 GiB states: n = 33 complex128 and n = 34 complex64.  Per-gate
    HBM bandwidth on a spread of targets and control/target pairs, then a
    500-gate random circuit followed by a QFT on all qubits (run fused)."""
    out = {}
    stream = torch.cuda.current_stream()
    for n, name in ((33, "c128"), (34, "c64")):
        dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
        S = (1 << n) * (16 if name == "c128" else 8)
        log(f"[bench] large: n={n} {name} ({S / 2**30:.0f} GiB)")
        st = Q.State(n, dtype, stream=stream)
        u, pairs = C.workload_sweep(n, 8, C.SEED_BASE + 2)
        one = {}
        for k in (0, 1, 5, 6, 7, 8, 12, 20, 27, n - 1):
            t = timed(lambda: st.apply_1q(k, u), stream, 3)
            one[str(k)] = round(2 * S / t / 1e9, 1)
        cu = {}
        for c, t_ in [(0, 1), (2, 20), (3, 20), (10, 0), (20, 10), (n - 1, 5)] + pairs[:4]:
            t = timed(lambda: st.apply_cu(c, t_, u), stream, 3)
            cu[f"{c},{t_}"] = round(S / t / 1e9, 1)
        # the top of the fused-vs-unfused sweep on this state: QFT and IQFT
        # fused, and the QFT with one streaming pass per gate
        top = {}
        for cname, qc in (("qft", C.qft_circuit(n)), ("iqft", C.iqft_circuit(n))):
            pg = sum((S if op["kind"] == C.OP_CU else 2 * S) for op in qc.ops)
            qi, _, _ = Q.qs_plan(n, dtype, qc.ops)
            tf = timed(lambda: st.run(qc.ops), stream, 1, warm=TUNE_CALLS)
            top[cname] = {"gates": len(qc), "passes_fused": qi["passes"], "fused_s": round(tf, 4),
                          "fused_hbm_GBps": round(qi["hbm_bytes"] / tf / 1e9, 1),
                          "fused_effective_GBps": round(pg / tf / 1e9, 1)}
            if cname == "qft":
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st.run(qc.ops, fuse=False)
                torch.cuda.synchronize()
                tu = time.perf_counter() - t0
                top[cname].update({"unfused_s": round(tu, 3), "unfused_effective_GBps": round(pg / tu / 1e9, 1),
                                   "speedup": round(tu / tf, 1)})
        log(f"[bench] large: n={n} {name} QFT/IQFT fused and unfused done")
        circ = C.workload_circuit_qft(n)
        info, _, _ = Q.qs_plan(n, dtype, circ.ops)
        pergate = sum((S if op["kind"] == C.OP_CU else 2 * S) for op in circ.ops)
        tc = timed(lambda: st.run(circ.ops), stream, 1, warm=TUNE_CALLS)
        winfo, _, _ = Q.qs_plan(n, dtype, circ.ops, flags=Q.QS_RUN_WIDE_TILES)
        tw = timed(lambda: st.run(circ.ops, wide=True), stream, 1, warm=TUNE_CALLS)
        qft = C.qft_circuit(n)
        qinfo, _, _ = Q.qs_plan(n, dtype, qft.ops)
        tq = timed(lambda: st.run(qft.ops), stream, 1, warm=TUNE_CALLS)
        out[f"n{n}_{name}"] = {
            "state_bytes": S,
            "one_qubit_GBps_by_target": one,
            "one_qubit_GBps_min": min(one.values()),
            "cu_alg_GBps": cu,
            "circuit": {"gates": len(circ), "passes": info["passes"], "s": round(tc, 4),
                        "hbm_GBps": round(info["hbm_bytes"] / tc / 1e9, 1),
                        "effective_GBps_paper_def": round(pergate / tc / 1e9, 1),
                        "paper_qft_only_s": {"33": 245.0, "34": 297.4}[str(n)],
                        "wide_tiles": {"passes": winfo["passes"], "s": round(tw, 4),
                                       "hbm_GBps": round(winfo["hbm_bytes"] / tw / 1e9, 1)}},
            "qft_iqft_fused_vs_unfused": top,
            "qft_only": {"gates": len(qft), "passes": qinfo["passes"], "s": round(tq, 4),
                         "effective_GBps_paper_def": round(
                             sum((S if op["kind"] == C.OP_CU else 2 * S) for op in qft.ops) / tq / 1e9, 1)},
        }
        del st
        torch.cuda.empty_cache()
    return out


def qft_section(Q, C, np, torch):
    """QFT and IQFT on all qubits, run fused (one HBM round trip per pass of
    gates) and with one streaming pass per gate, over a sweep of widths: the
    GPU analogue of the paper's fused-vs-unfused comparison (Sec. 5.5).
    Effective bandwidth is the paper's definition: the per-gate algorithmic
    bytes (Table 2: 2S per 1q gate, S per controlled gate) over the time."""
    out = {}
    stream = torch.cuda.current_stream()
    for name, dtype, b, ns in (("c128", Q.QS_C128, 16, (18, 20, 22, 24, 26, 28, 30, 31, 32)),
                               ("c64", Q.QS_C64, 8, (19, 21, 23, 25, 27, 29, 31, 32, 33))):
        rows = {}
        for n in ns:
            S = (1 << n) * b
            st = Q.State(n, dtype, stream=stream)
            rec = {}
            for cname, circ in (("qft", C.qft_circuit(n)), ("iqft", C.iqft_circuit(n))):
                pergate = sum((S if op["kind"] == C.OP_CU else 2 * S) for op in circ.ops)
                info, _, _ = Q.qs_plan(n, dtype, circ.ops)
                reps = 3 if n <= 24 else 1
                tf = timed(lambda: st.run(circ.ops), stream, reps, warm=TUNE_CALLS)
                rec[cname] = {
                    "gates": len(circ), "passes_fused": info["passes"], "fused_s": round(tf, 5),
                    "fused_effective_GBps": round(pergate / tf / 1e9, 1),
                    "fused_hbm_GBps": round(info["hbm_bytes"] / tf / 1e9, 1),
                }
                # above 2^30 amplitudes the unfused leg (one streaming pass per
                # gate, seconds) is timed once, for the QFT only
                if n <= 30 or cname == "qft":
                    if n <= 30:
                        tu = timed(lambda: st.run(circ.ops, fuse=False), stream, reps)
                    else:
                        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        e0.record(stream)
                        st.run(circ.ops, fuse=False)
                        e1.record(stream)
                        e1.synchronize()
                        tu = e0.elapsed_time(e1) * 1e-3
                    rec[cname].update({"unfused_s": round(tu, 5),
                                       "unfused_effective_GBps": round(pergate / tu / 1e9, 1),
                                       "speedup": round(tu / tf, 2)})
            rows[str(n)] = rec
            del st
            torch.cuda.empty_cache()
        log(f"[bench] qft sweep {name}: n={ns[0]}..{ns[-1]} done")
        out[name] = rows
    return out


def kq_section(Q, C, np, torch, n):
    """Dense gates on k = 1..5 qubits (qs_apply_kq) on the n-qubit complex128
    state: HBM bandwidth (2 * 2^n * 16 bytes per gate) and FP64 rate (8 * 2^k
    flop per amplitude) for the lowest, the highest and spread-out target
    sets."""
    out = {}
    stream = torch.cuda.current_stream()
    S = (1 << n) * 16
    st = Q.State(n, Q.QS_C128, stream=stream)
    rng = np.random.default_rng(C.SEED_BASE + 5)
    for k in range(1, Q.QS_KQ_MAX + 1):
        dim = 1 << k
        z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / np.sqrt(2)
        u, _ = np.linalg.qr(z)
        rec = {}
        for label, targets in (("low", list(range(k))), ("high", list(range(n - k, n))),
                               ("spread", [int(round(j * (n - 1) / max(1, k - 1))) for j in range(k)])):
            t = timed(lambda: st.apply_kq(targets, u), stream, 3)
            rec[label] = {"targets": targets, "ms": round(t * 1e3, 3), "GBps": round(2 * S / t / 1e9, 1),
                          "TFLOPs": round(8 * dim * (1 << n) / t / 1e12, 2)}
        out[f"k{k}"] = rec
    del st
    torch.cuda.empty_cache()
    log(f"[bench] k-qubit gates n={n}: done")
    return out


def reorder_section(Q, C, np, torch, n):
    """Qubit reordering (Sec. 6) on the n-qubit complex128 state.  The
    permutation kernels: swaps of upper qubits move only the 1 KiB blocks
    that change place, 2 (1 - 2^-k) S bytes for k swaps; a swap that touches
    a block bit moves 2 S.  Then the reordered runner for a state split by
    its top 3 qubits (8 shards), against the plain run of the same circuits:
    the reorderings it inserts and the network traffic per shard with them
    and with Sec. 3.2's pairwise exchanges (Table 2's counts)."""
    out = {"permute": {}, "runs": {}}
    stream = torch.cuda.current_stream()
    S = (1 << n) * 16
    st = Q.State(n, Q.QS_C128, stream=stream)

    def swaps(pairs):
        p = list(range(n))
        for a, b in pairs:
            p[a], p[b] = b, a
        return p

    cases = (("one_upper_swap", swaps([(n - 1, 9)]), 2 * 0.5 * S),
             ("three_upper_swaps", swaps([(n - 1, 9), (n - 2, 8), (n - 3, 7)]), 2 * 0.875 * S),
             ("block_bit_swap", swaps([(0, n - 1)]), 2 * S),
             ("reverse", list(range(n))[::-1], None))
    for label, perm, nbytes in cases:
        t = timed(lambda: st.permute_qubits(perm), stream, 4)
        rec = {"ms": round(t * 1e3, 3)}
        if nbytes:
            rec["bytes"] = nbytes
            rec["GBps"] = round(nbytes / t / 1e9, 1)
        out["permute"][label] = rec
    for label, ops in (("random1000", C.random_circuit(n, 1000, np.random.default_rng(C.SEED_BASE + 1)).ops),
                       ("random500_qft", C.workload_circuit_qft(n, 500).ops)):
        t_plain = timed(lambda: st.run(ops), stream, 1, warm=TUNE_CALLS)
        info = {}

        def reordered():
            info.update(st.run_reordered(ops, n - 3))

        t_re = timed(reordered, stream, 1, warm=TUNE_CALLS)
        out["runs"][label] = {"plain_ms": round(t_plain * 1e3, 1), "reordered_ms": round(t_re * 1e3, 1),
                              "upper_qubits": 3, **info}
    del st
    torch.cuda.empty_cache()
    log(f"[bench] qubit reordering n={n}: done")
    return out


def adjoint_section(Q, C, np, torch, ps_pairs):
    """Energy + full gradient of the layered ansatz (L = 20, H = 100 Pauli
    strings) by the adjoint method vs the 2P-sweep parameter-shift rule on the
    same GPU, FP64 (complex128) state."""
    out = {}
    stream = torch.cuda.current_stream()
    for n in (20, 28):
        circ, ham = C.workload_ansatz(n, 20, 100)
        P = circ.nparams
        x, z = Q.pauli_masks(ham.codes)
        st = Q.State(n, Q.QS_C128, stream=stream)
        lam = Q.State(n, Q.QS_C128, stream=stream, init=False)
        log(f"[bench] adjoint: n={n}, P={P}, gates={len(circ)}")

        def adj():
            st.init_basis(0)
            return Q.qs_grad_adjoint(st.handle, circ.ops, circ.theta, x, z, ham.coeff, lam.handle)

        for _ in range(TUNE_CALLS):  # compile, then every tile order timed
            adj()
            torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3 if n == 20 else 1
        for _ in range(reps):
            e, g = adj()
        t_adj = (time.perf_counter() - t0) / reps

        def energy(th):
            st.init_basis(0)
            st.run(circ.ops, th)
            return Q.qs_expect_pauli(st.handle, x, z, ham.coeff)

        pairs = P if n == 20 else min(ps_pairs, P)
        for _ in range(TUNE_CALLS):  # tile orders timed before the timed loop
            energy(circ.theta)
            torch.cuda.synchronize()
        t0 = time.perf_counter()
        gps = np.zeros(pairs)
        for j in range(pairs):
            tp = circ.theta.copy()
            tm = circ.theta.copy()
            tp[j] += np.pi / 2
            tm[j] -= np.pi / 2
            gps[j] = 0.5 * (energy(tp) - energy(tm))
        t_pairs = time.perf_counter() - t0
        t_ps = t_pairs * P / pairs
        rec = {
            "params": P, "gates": len(circ), "terms": 100,
            "adjoint_s": round(t_adj, 4), "param_shift_s": round(t_ps, 3),
            "param_shift_pairs_timed": pairs,
            "param_shift_extrapolated": pairs < P,
            "speedup": round(t_ps / t_adj, 1),
            "max_abs_diff_adjoint_vs_shift": float(np.abs(g[:pairs] - gps).max()),
            "energy": e,
        }
        del st, lam
        torch.cuda.empty_cache()
        # the same energy and gradient on a complex64 state (FP64 accumulation)
        s64 = Q.State(n, Q.QS_C64, stream=stream)
        l64 = Q.State(n, Q.QS_C64, stream=stream, init=False)

        def adj64():
            s64.init_basis(0)
            return Q.qs_grad_adjoint(s64.handle, circ.ops, circ.theta, x, z, ham.coeff, l64.handle)

        adj64()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            e64, g64 = adj64()
        rec["c64_adjoint_s"] = round((time.perf_counter() - t0) / reps, 4)
        if n == 28:
            # the two sweeps apart, for per-pass rooflines
            s128 = Q.State(n, Q.QS_C128, stream=stream)
            l128 = Q.State(n, Q.QS_C128, stream=stream, init=False)
            rec["sweeps"] = {
                "c128": sweep_split(Q, torch, np, n, circ, x, z, ham.coeff, Q.QS_C128, s128, l128, stream),
                "c64": sweep_split(Q, torch, np, n, circ, x, z, ham.coeff, Q.QS_C64, s64, l64, stream)}
            del s128, l128
            torch.cuda.empty_cache()
            # both sweeps on wide tiles (fewer passes), complex128 and complex64
            for nm, s_, l_ in (("c128", None, None), ("c64", s64, l64)):
                if s_ is None:
                    s_ = Q.State(n, Q.QS_C128, stream=stream)
                    l_ = Q.State(n, Q.QS_C128, stream=stream, init=False)

                def adjw():
                    s_.init_basis(0)
                    return Q.qs_grad_adjoint(s_.handle, circ.ops, circ.theta, x, z, ham.coeff, l_.handle,
                                             Q.QS_ADJ_WIDE_TILES)

                adjw()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ew, gw = adjw()
                rec[f"{nm}_adjoint_wide_tiles_s"] = round(time.perf_counter() - t0, 4)
                ref_e, ref_g = (e, g) if nm == "c128" else (e64, g64)
                rec[f"{nm}_wide_tiles_max_abs_diff"] = {"energy": abs(ew - ref_e), "gradient": float(np.abs(gw - ref_g).max())}
                del s_, l_
                torch.cuda.empty_cache()
        rec["c64_max_abs_diff_vs_c128"] = {"energy": abs(e64 - e), "gradient": float(np.abs(g64 - g).max())}
        del s64, l64
        torch.cuda.empty_cache()
        if n == 20:
            rec["error_vs_fp64_oracle"] = oracle_errors(C, np, circ, ham, n, {"c128": (e, g), "c64": (e64, g64)})
        out[f"n{n}"] = rec
    return out


def sweep_split(Q, torch, np, n, circ, x, z, coeff, dtype, st, lam, stream, reps=3):
    """The adjoint's forward sweep (a fused run of the circuit), lambda = H psi
    alone, and H psi + energy + reverse sweep (QS_ADJ_STATE_IS_FINAL on the
    final state), each timed; the reverse sweep is the last minus H psi.
    Per-pass times against 2S (forward) and 4S (reverse, psi and lambda)."""
    S = (1 << n) * (16 if dtype == Q.QS_C128 else 8)
    fwd, _, _ = Q.qs_plan(n, dtype, circ.ops, circ.theta)
    rev, _, _ = Q.qs_plan(n, dtype, circ.ops, circ.theta, flags=Q.QS_PLAN_ADJOINT_REVERSE)
    tf, th, tr = [], [], []
    for i in range(reps + TUNE_CALLS):
        st.init_basis(0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st.run(circ.ops, circ.theta)
        e1.record(stream)
        Q.qs_apply_pauli_sum(st.handle, lam.handle, x, z, coeff)
        e2.record(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Q.qs_grad_adjoint(st.handle, circ.ops, circ.theta, x, z, coeff, lam.handle, Q.QS_ADJ_STATE_IS_FINAL)
        t1 = time.perf_counter()
        if i >= TUNE_CALLS:  # the first rounds compile and time the tile orders
            tf.append(e0.elapsed_time(e1) * 1e-3)
            th.append(e1.elapsed_time(e2) * 1e-3)
            tr.append(t1 - t0)
    f_s, h_s, fin_s = (float(np.median(v)) for v in (tf, th, tr))
    r_s = fin_s - h_s
    fp, rp = f_s / fwd["passes"], r_s / rev["passes"]
    return {"forward_passes": fwd["passes"], "forward_s": round(f_s, 4), "forward_pass_ms": round(fp * 1e3, 4),
            "forward_pass_frac": round(2 * S / fp / 1e9 / PEAK_HBM_GBPS, 4),
            "h_psi_s": round(h_s, 4), "final_state_adjoint_s": round(fin_s, 4),
            "reverse_passes": rev["passes"], "reverse_s": round(r_s, 4), "reverse_pass_ms": round(rp * 1e3, 4),
            "reverse_pass_frac": round(4 * S / rp / 1e9 / PEAK_HBM_GBPS, 4)}


def oracle_errors(C, np, circ, ham, n, results, nsample=8):
    """Energy and sampled-gradient errors of GPU results against the FP64
    CPU oracle (its energy, and its parameter-shift rule on `nsample`
    parameters spread over the circuit, first and last included)."""
    import oracle as O
    O.set_threads(min(16, os.cpu_count() or 1))
    P = circ.nparams
    params = sorted({int(round(j * (P - 1) / (nsample - 1))) for j in range(nsample)})
    t0 = time.perf_counter()
    re = O.energy(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    rg = O.grad_param_shift(circ.ops, n, circ.theta, ham.codes, ham.coeff, params=params)
    out = {"params_checked": params, "oracle_s": round(time.perf_counter() - t0, 2)}
    for k, (e, g) in results.items():
        out[k] = {"energy_abs_err": abs(e - re), "gradient_max_abs_err": float(np.abs(g[params] - rg[params]).max())}
    return out


def batch_section(Q, C, np, torch):
    """4096 independent ansatz circuits (n uniform in 10..18, L in 5..30, 20
    Pauli strings each): energy + full adjoint gradient of all of them in one
    persistent launch (qs_batch_run), complex128 and complex64, with the
    launch shape chosen by the autotuner on the batch itself.  Compared
    with one qs_grad_adjoint call per circuit on the same GPU (timed on every
    64th circuit, extrapolated)."""
    from paper_1601_07195_amd import autotune as A
    wl = C.workload_batch(4096)
    items = [(c.n, c.ops, c.theta, h.codes, h.coeff) for c, h in wl]
    nparams = sum(len(i[2]) for i in items)
    # LDS traffic model of the kernel: every gate reads and writes each
    # amplitude of psi once forward and of psi and lambda once in reverse
    upd = sum(len(i[1]) * (1 << i[0]) * 3 for i in items)
    out = {"circuits": len(items), "gates": sum(len(i[1]) for i in items), "params": nparams}
    ref = None
    for dt, name, ab in ((Q.QS_C128, "c128", 16), (Q.QS_C64, "c64", 8)):
        t0 = time.perf_counter()
        b = Q.Batch(items, dt)
        t_create = time.perf_counter() - t0
        tune = A.tune(b, repeats=1)
        shape = A.fields(tune)
        log(f"[bench] batch {name}: tuned {shape}")
        # each shape is timed on its own run of calls: a change of the LDS
        # chunk shape rebuilds the host schedule, which is not kernel time
        times, times_def = [], []
        b.run_flat(A.DEFAULT)
        for _ in range(3):
            t0 = time.perf_counter()
            b.run_flat(A.DEFAULT)
            times_def.append(time.perf_counter() - t0)
        b.run_flat(shape)
        for _ in range(3):
            t0 = time.perf_counter()
            e, g = b.run_flat(shape)
            times.append(time.perf_counter() - t0)
        t_b = statistics.median(times)
        idx = list(range(0, len(items), 64))
        t0 = time.perf_counter()
        for i in idx:
            n, ops, th, codes, coeff = items[i]
            st = Q.State(n, dt)
            lam = Q.State(n, dt, init=False)
            Q.grad_adjoint(st, lam, ops, th, codes, coeff)
        torch.cuda.synchronize()
        t_un = (time.perf_counter() - t0) * len(items) / len(idx)
        rec = {
            "create_s": round(t_create, 3), "tuning": shape,
            "batch_s": round(t_b, 4), "batch_default_shape_s": round(statistics.median(times_def), 4),
            "circuits_per_s": round(len(items) / t_b, 1),
            "gradient_entries_per_s": round(nparams / t_b, 1),
            "unbatched_s_extrapolated": round(t_un, 3), "unbatched_circuits_timed": len(idx),
            "speedup_vs_unbatched": round(t_un / t_b, 1),
            "lds_bytes_model": upd * 2 * ab,
            "lds_GBps_model": round(upd * 2 * ab / t_b / 1e9, 1),
        }
        if ref is None:
            ref = (e, g)
        else:
            rec["max_abs_diff_vs_c128"] = {"energy": float(np.abs(e - ref[0]).max()),
                                           "gradient": float(np.abs(g - ref[1]).max())}
        rec["error_vs_fp64_oracle"] = batch_oracle_errors(C, np, items, e, g)
        out[name] = rec
        b.close()
    return out


def batch_oracle_errors(C, np, items, e, g, nsample=8):
    """Errors of batched results against the FP64 CPU oracle on a seeded
    sample of circuits (the widest-deepest and the deepest among them):
    energies, and the parameter-shift gradient on six parameters each."""
    import oracle as O
    O.set_threads(min(16, os.cpu_count() or 1))
    ns = np.array([it[0] for it in items])
    depth = np.array([len(it[1]) for it in items])
    pick = [int(np.argmax(depth + (ns == ns.max()) * 10 ** 6)), int(np.argmax(depth))]
    for i in np.random.default_rng(4096).choice(len(items), nsample, replace=False):
        if int(i) not in pick:
            pick.append(int(i))
    pick = pick[:nsample]
    off = np.concatenate([[0], np.cumsum([len(it[2]) for it in items])])
    worst_e = worst_g = 0.0
    t0 = time.perf_counter()
    for i in pick:
        n, ops, th, codes, coeff = items[i]
        P = len(th)
        params = sorted({0, 1, n, P // 2, P - n - 1, P - 1})
        re = O.energy(ops, n, th, codes, coeff)
        rg = O.grad_param_shift(ops, n, th, codes, coeff, params=params)
        gi = np.asarray(g[off[i]:off[i + 1]])
        worst_e = max(worst_e, abs(float(e[i]) - re))
        worst_g = max(worst_g, float(np.abs(gi[params] - rg[params]).max()))
    return {"circuits": pick, "qubits": [int(items[i][0]) for i in pick],
            "energy_max_abs_err": worst_e, "gradient_max_abs_err": worst_g,
            "oracle_s": round(time.perf_counter() - t0, 2)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(the simulator holds the whole state on one GPU).", file=sys.stderr)
        sys.exit(2)
    if args.workload_only:
        workload_only(args)
        return

    import numpy as np
    import torch

    import circuits as C
    import paper_1601_07195_amd.qs as Q

    torch.cuda.set_device(0)
    n = args.n
    dtype = Q.QS_C128 if args.dtype == "c128" else Q.QS_C64
    b = 16 if dtype == Q.QS_C128 else 8
    S = (1 << n) * b
    seed = C.SEED_BASE + 1
    u, pairs = C.workload_sweep(n, args.ncu, seed)
    circ = C.random_circuit(n, args.circuit_gates, np.random.default_rng(seed))
    log(f"[bench] n={n} {args.dtype} state {S / 2**30:.1f} GiB, steps={args.steps} warmup={args.warmup}")

    stream = torch.cuda.current_stream()
    st = Q.State(n, dtype, stream=stream)
    timer = EventTimer(stream)

    # algorithmic bytes of one step
    n_cu_alg = len(pairs)
    bytes_sweep_1q = 2 * n * 2 * S
    bytes_cu = n_cu_alg * S
    # per-gate (Table 2) bytes of the circuit, and the HBM bytes of the
    # passes the fusion planner actually runs
    bytes_circ_pergate = sum((S if op["kind"] == C.OP_CU else 2 * S) for op in circ.ops)
    plan_info, _, _ = Q.qs_plan(n, dtype, circ.ops)
    bytes_circ = plan_info["hbm_bytes"]
    bytes_probs = S
    step_bytes = bytes_sweep_1q + bytes_cu + bytes_circ + bytes_probs

    def step(record: bool):
        for k in range(n):
            if record:
                timer.measure(("h", k), lambda: st.apply_1q(k, C.H_GATE))
                timer.measure(("u", k), lambda: st.apply_1q(k, u))
            else:
                st.apply_1q(k, C.H_GATE)
                st.apply_1q(k, u)
        for c, t in pairs:
            if record:
                timer.measure(("cu", c, t), lambda: st.apply_cu(c, t, u))
            else:
                st.apply_cu(c, t, u)
        if record:
            timer.measure(("circuit",), lambda: st.run(circ.ops))
            timer.measure(("probs",), lambda: st.probabilities())
        else:
            st.run(circ.ops)
            st.probabilities()

    # compiled passes time each tile order on one of their first launches
    # and keep the fastest: untimed runs of the circuit before the warmup
    for _ in range(TUNE_CALLS):
        st.run(circ.ops)
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        log(f"[bench] step {i + 1}/{args.steps} queued")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    durations = timer.collect()
    ms_per_step = elapsed / args.steps * 1e3
    value = step_bytes * args.steps / elapsed / 1e9

    one_q = [d for k, v in durations.items() if k[0] in ("h", "u") for d in v]
    per_target = {}
    for k, v in durations.items():
        if k[0] in ("h", "u"):
            per_target.setdefault(k[1], []).extend(v)
    cu_t = [d for k, v in durations.items() if k[0] == "cu" for d in v]
    # controls inside a 128-byte line (unit bit < 3: control qubit < 3 at
    # complex128, < 4 at complex64) make every line hold both halves, so the
    # hardware moves the whole state: at most half the peak in algorithmic
    # bytes.  Reported apart from the other pairs.
    line_bits = 3 if args.dtype == "c128" else 4
    cu_low = [d for k, v in durations.items() if k[0] == "cu" and k[1] < line_bits for d in v]
    cu_reg = [d for k, v in durations.items() if k[0] == "cu" and k[1] >= line_bits for d in v]
    circ_t = durations[("circuit",)]
    probs_t = durations[("probs",)]
    mean_1q = statistics.fmean(one_q)
    achieved = 2 * S / mean_1q / 1e9
    tgt_gbps = {k: 2 * S / statistics.median(v) / 1e9 for k, v in per_target.items()}
    cu_gbps = sorted(S / d / 1e9 for d in cu_t)

    # the same circuit with wide tiles (fewer low qubits fixed per tile:
    # fewer passes, each at a lower fraction of peak)
    wide_info, _, _ = Q.qs_plan(n, dtype, circ.ops, flags=Q.QS_RUN_WIDE_TILES)
    t_wide = timed(lambda: st.run(circ.ops, wide=True), stream, 3, warm=TUNE_CALLS)

    # STREAM copy (B_mem, Sec. 5.2) on a 2 x 4 GiB pair of buffers
    cs = 4 << 30
    src = torch.empty(cs // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    Q.qs_stream_copy(src, dst)
    torch.cuda.synchronize()
    reps = 10
    for _ in range(reps):
        timer.measure(("copy",), lambda: Q.qs_stream_copy(src, dst))
    torch.cuda.synchronize()
    copy_t = timer.collect()[("copy",)]
    copy_gbps = 2 * cs / statistics.median(copy_t) / 1e9
    del src, dst

    # per-kernel rooflines; the dominant kernel (most time in a step) is
    # reported as `roofline`.  Fused passes: the circuit's event-timed
    # duration divided by its launches (all fused for this circuit).
    n_sweep = len(one_q) / args.steps
    circ_med = statistics.median(circ_t)
    # fused passes run compiled per pass shape from n = 26 (the library's
    # automatic choice), on the interpreter kernels below that
    fused_name = ("qs_pass_* (fused pass compiled for its shape, circuit)" if n >= 26
                  else "k_fused (interpreted fused pass, circuit)")
    kernels = {
        fused_name: {
            "launches_per_step": plan_info["passes"], "bytes_per_launch": 2 * S,
            "mean_launch_ms": circ_med / plan_info["passes"] * 1e3,
            "step_s": circ_med},
        "k_exchange/k_pair (single-qubit gate, streaming)": {
            "launches_per_step": n_sweep, "bytes_per_launch": 2 * S,
            "mean_launch_ms": mean_1q * 1e3, "step_s": mean_1q * n_sweep},
        "k_exchange/k_pair (controlled gate, streaming)": {
            "launches_per_step": len(pairs), "bytes_per_launch": S,
            "mean_launch_ms": statistics.fmean(cu_t) * 1e3,
            "step_s": statistics.fmean(cu_t) * len(pairs)},
    }
    if cu_reg:
        kernels["k_exchange/k_pair (controlled gate, control outside the 128-byte line)"] = {
            "launches_per_step": len(cu_reg) / args.steps, "bytes_per_launch": S,
            "mean_launch_ms": statistics.fmean(cu_reg) * 1e3,
            "step_s": statistics.fmean(cu_reg) * len(cu_reg) / args.steps}
    # HBM traffic per launch of the streamed gates, from their counter summary
    gkeys = {"k_exchange/k_pair (single-qubit gate, streaming)": "one_qubit",
             "k_exchange/k_pair (controlled gate, streaming)": "cu_all",
             "k_exchange/k_pair (controlled gate, control outside the 128-byte line)": "cu_outside_line"}
    for k, key in gkeys.items():
        if k in kernels:
            kernels[k]["traffic"] = measured_traffic("k_pair_k_exchange_gates", f"{args.dtype}_n{n}", key)
    for v in kernels.values():
        v["achieved_GBps"] = round(v["bytes_per_launch"] / (v["mean_launch_ms"] * 1e-3) / 1e9, 1)
        v["frac"] = round(v["achieved_GBps"] / PEAK_HBM_GBPS, 4)
        v["mean_launch_ms"] = round(v["mean_launch_ms"], 4)
        v["step_s"] = round(v["step_s"], 4)
    if n >= 26:  # the compiled passes' summary
        kernels[fused_name]["traffic"] = measured_traffic(f"qs_pass_compiled_circuit_{args.dtype}", f"n{n}")
    dom = max(kernels, key=lambda k: kernels[k]["step_s"])
    traffic = kernels[dom].get("traffic")
    roof = {"kernel": dom, "bound": "hbm", "achieved": kernels[dom]["achieved_GBps"],
            "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": kernels[dom]["frac"], "traffic": traffic,
            "bytes_per_launch": kernels[dom]["bytes_per_launch"],
            "mean_launch_ms": kernels[dom]["mean_launch_ms"]}

    line = {
        "metric": "gate HBM GB/s (% peak) at n=30-34; adjoint grad s vs parameter-shift, same GPU",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if dtype == Q.QS_C128 else "f32",
        "data": "synthetic (seeded Haar-random gates)",
        "config": {
            "workload": f"per-gate sweep n={n} {args.dtype}: H and Haar U on every target, "
                        f"controlled-U on {len(pairs)} random pairs, {args.circuit_gates}-gate random "
                        f"circuit, per-qubit probabilities",
            "n": n, "state_bytes": S, "parallelism": "single GPU",
        },
        "pct_peak": round(100 * value / PEAK_HBM_GBPS, 1),
        "roofline": roof,
        "roofline_by_kernel": kernels,
        "detail": {
            "one_qubit_GBps_by_target": {str(k): round(v, 1) for k, v in sorted(tgt_gbps.items())},
            "one_qubit_GBps_min": round(min(tgt_gbps.values()), 1),
            "cu_GBps_control_outside_line": round(S / statistics.fmean(cu_reg) / 1e9, 1) if cu_reg else None,
            "cu_GBps_control_inside_line": round(S / statistics.fmean(cu_low) / 1e9, 1) if cu_low else None,
            "cu_pairs_control_inside_line": len(cu_low) // max(1, args.steps),
            "cu_GBps_min_median_max": [round(cu_gbps[0], 1), round(statistics.median(cu_gbps), 1),
                                       round(cu_gbps[-1], 1)],
            "circuit_ms": round(statistics.median(circ_t) * 1e3, 3),
            "circuit_passes": plan_info["passes"],
            "circuit_fused_passes": plan_info["fused"],
            "circuit_hbm_GBps": round(bytes_circ / statistics.median(circ_t) / 1e9, 1),
            "circuit_effective_GBps_paper_def": round(bytes_circ_pergate / statistics.median(circ_t) / 1e9, 1),
            "circuit_wide_tiles": {"ms": round(t_wide * 1e3, 3), "passes": wide_info["passes"],
                                   "hbm_GBps": round(wide_info["hbm_bytes"] / t_wide / 1e9, 1),
                                   "pass_frac": round(wide_info["hbm_bytes"] / t_wide / 1e9 / PEAK_HBM_GBPS, 4)},
            "probabilities_GBps": round(S / statistics.median(probs_t) / 1e9, 1),
        },
        "stream_copy": {"GBps": round(copy_gbps, 1), "bytes": 2 * cs,
                        "gate_1q_vs_copy": round(achieved / copy_gbps, 3)},
        "paper_context": "qHiPSTER (Stampede, 1 Xeon E5-2680 socket, complex128, n=29): 1q gate "
                         "0.44 s measured vs 0.43 s bound = 39 GB/s vs STREAM 40 GB/s (Table 2, Sec. 5.4)",
    }
    del st
    torch.cuda.empty_cache()
    if not args.no_large:
        line["large_states"] = large_section(Q, C, np, torch)
    if not args.no_qft:
        line["qft_fused_vs_unfused"] = qft_section(Q, C, np, torch)
    if not args.no_kq:
        line["kq_gates"] = kq_section(Q, C, np, torch, n)
    if not args.no_reorder:
        line["qubit_reordering"] = reorder_section(Q, C, np, torch, n)
    if not args.no_adjoint:
        line["adjoint_vs_param_shift"] = adjoint_section(Q, C, np, torch, args.ps_pairs)
    if not args.no_batch:
        line["batch"] = batch_section(Q, C, np, torch)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle sample")
        line["cpu_baseline"] = cpu_baseline(n, u, pairs, args)
    js = Q.qs_get_jit_stats()
    line["compiled_passes"] = {
        "kernels_compiled": js["kernels_compiled"], "compile_s_total": round(js["compile_seconds"], 2),
        "programs_clang": js["programs_clang"], "programs_hiprtc": js["programs_hiprtc"],
        "note": "fused passes at n >= 26 run kernels compiled per pass shape; compiled during warmup "
                "and the untimed first call of each section, never inside a timed region"}
    line["roofline_by_kernel"].update(section_rooflines(line))
    line["precision_summary"] = precision_summary(line)
    line["per_gate_summary"] = per_gate_summary(line, n, args.dtype, S)
    print(json.dumps(line), flush=True)


def precision_summary(line: dict) -> dict:
    """Errors against the FP64 CPU oracle of the energy / gradient results:
    the n = 20 ansatz (L = 20, 100 strings) and the 4096-circuit batch
    (sampled circuits), complex128 and complex64 states."""
    out = {}
    a = line.get("adjoint_vs_param_shift", {}).get("n20", {}).get("error_vs_fp64_oracle")
    if a:
        out["ansatz_n20"] = {k: a[k] for k in ("c128", "c64") if k in a}
    b = line.get("batch", {})
    for k in ("c128", "c64"):
        if k in b and "error_vs_fp64_oracle" in b[k]:
            r = b[k]["error_vs_fp64_oracle"]
            out.setdefault("batch_4096", {})[k] = {"energy_abs_err": r["energy_max_abs_err"],
                                                  "gradient_max_abs_err": r["gradient_max_abs_err"]}
    return out


def per_gate_summary(line: dict, n: int, dtype: str, S: int) -> dict:
    """The figures the per-gate HBM claim rests on, for n = 30, 33 and 34,
    gathered from the sections above (GB/s of algorithmic bytes, and the
    fraction of the 8 TB/s peak)."""
    def frac(v):
        return None if v is None else round(v / PEAK_HBM_GBPS, 3)
    d = line["detail"]
    one = list(d["one_qubit_GBps_by_target"].values())
    out = {f"n{n}_{dtype}": {
        "one_qubit_min_GBps": round(min(one), 1), "one_qubit_median_GBps": round(statistics.median(one), 1),
        "cu_control_outside_line_GBps": d["cu_GBps_control_outside_line"],
        "cu_control_inside_line_GBps": d["cu_GBps_control_inside_line"],
        "fused_circuit_hbm_GBps": d["circuit_hbm_GBps"],
        "fused_pass_frac": line["roofline"]["frac"],
    }}
    q = line.get("qft_fused_vs_unfused", {}).get("c128", {}).get(str(n))
    if q:
        out[f"n{n}_{dtype}"]["qft_fused_hbm_GBps"] = q["qft"]["fused_hbm_GBps"]
        out[f"n{n}_{dtype}"]["iqft_fused_hbm_GBps"] = q["iqft"]["fused_hbm_GBps"]
    for key, rec in line.get("large_states", {}).items():
        lb = 3 if key.endswith("c128") else 4
        cu_in = [v for k, v in rec["cu_alg_GBps"].items() if int(k.split(",")[0]) < lb]
        cu_out = [v for k, v in rec["cu_alg_GBps"].items() if int(k.split(",")[0]) >= lb]
        o1 = list(rec["one_qubit_GBps_by_target"].values())
        qo = rec["qft_only"]
        Sx = rec["state_bytes"]
        out[key] = {
            "one_qubit_min_GBps": round(min(o1), 1), "one_qubit_median_GBps": round(statistics.median(o1), 1),
            "cu_control_outside_line_GBps": round(statistics.fmean(cu_out), 1) if cu_out else None,
            "cu_control_inside_line_GBps": round(statistics.fmean(cu_in), 1) if cu_in else None,
            "fused_circuit_hbm_GBps": rec["circuit"]["hbm_GBps"],
            "qft_per_pass_hbm_GBps": round(qo["passes"] * 2 * Sx / qo["s"] / 1e9, 1),
        }
    for v in out.values():
        for k in list(v):
            if k.endswith("_GBps"):
                v[k.replace("_GBps", "_frac")] = frac(v[k])
    return out


if __name__ == "__main__":
    main()
