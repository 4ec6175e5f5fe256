"""Benchmark: energy + adjoint-gradient evaluations per second of the 24-qubit
workload (12 electrons, 200 sampled excitations, FP64) on one GPU, the HBM
roofline fraction of its dominant kernel (the adjoint packet run, each
launch's own start and end taken live), the per-parameter finite-difference
gradient on the same GPU, the FP32-amplitude variant, ADAPT screening, the
Strategy-2 loop, and the FP64 CPU oracle timed on the host cores; then the
30-qubit workload (14 electrons, 500 operators; FP64 and FP32 rates, its
dominant kernel's roofline, finite differences on 16 parameters extrapolated
to all of them).

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def qubit_of(so, m, ordering):
    p, s = divmod(int(so), 2)
    return int(so) if ordering == 0 else p + s * m


def line_bytes(op, n, amp_bytes, ordering):
    """Read + write of the 128-byte lines one pair kernel touches."""
    m = n // 2
    low = 3 if amp_bytes == 16 else 4
    qs = [qubit_of(v, m, ordering) for v in op if v >= 0]
    hi = sum(q >= low for q in qs)
    frac = 1.0 if hi == 0 else min(1.0, 2.0 ** (1 - hi))
    return 2.0 * (2 ** n) * amp_bytes * frac


def model_bytes(p, amp_bytes):
    """Dense line-granular model: each operator reads and writes the 128-byte
    lines holding its active amplitude pairs."""
    per_op = [line_bytes(op, p.n_qubits, amp_bytes, p.ordering) for op in p.ops]
    fwd = sum(per_op)
    sigma = 2.0 * (2 ** p.n_qubits) * amp_bytes
    return {"forward": fwd, "reverse": 2 * fwd, "sigma_floor": sigma, "eval": 3 * fwd + sigma,
            "per_op": per_op}


def sector_pairs(op, m, na, nb):
    """Active pairs of one operator on the (na, nb) sector: strings of each spin
    that hold its annihilated orbitals and lack its created ones."""
    from math import comb
    cnt = {0: [0, 0], 1: [0, 0]}  # spin -> [annihilated, created]
    a, b, j, i = (int(v) for v in op)
    for v in (i, j):
        if v >= 0:
            cnt[v % 2][0] += 1
    for v in (a, b):
        if v >= 0:
            cnt[v % 2][1] += 1
    out = 1
    for s, ne in ((0, na), (1, nb)):
        d, c = cnt[s]
        out *= comb(m - d - c, ne - d) if (d or c) else comb(m, ne)
    return out


def sector_model_bytes(p, amp_bytes):
    """Sector-compressed model: each operator reads and writes both amplitudes
    of every active sector pair (forward: psi; reverse: psi and lambda)."""
    m = p.n_orb
    per_op = [4.0 * amp_bytes * sector_pairs(op, m, p.n_alpha, p.n_beta) for op in p.ops]
    fwd = sum(per_op)
    from math import comb
    dim = comb(m, p.n_alpha) * comb(m, p.n_beta)
    sigma = 2.0 * dim * amp_bytes
    return {"forward": fwd, "reverse": 2 * fwd, "sigma_floor": sigma, "eval": 3 * fwd + sigma,
            "per_op": per_op}


def fd_subset(plan, p, g, psi, lam, n_params=16, h=1e-5):
    """Central finite differences on the first n_params angles.  Each energy
    is the forward sweep and H psi on the sector state (the stage calls, as
    the library's own finite-difference gradient does per energy); the time
    per energy is extrapolated to the 2K + 1 energies of a whole
    finite-difference gradient (labelled as an extrapolation)."""
    import torch
    th = np.array(p.theta, dtype=np.float64)

    def energy(t):
        plan.set_theta(t)
        plan.forward_async(psi)
        plan.sigma_async(psi, lam)
        return plan.finish()[0]

    energy(th)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gfd = np.zeros(n_params)
    for k in range(n_params):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        gfd[k] = (energy(tp) - energy(tm)) / (2 * h)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    per_energy = dt / (2 * n_params)
    full = per_energy * (2 * p.n_ops + 1)
    return {"params_measured": n_params, "measured_s": dt, "per_energy_ms": per_energy * 1e3,
            "extrapolated_full_fd_s": full, "extrapolated": True,
            "max_abs_diff_vs_adjoint_on_subset": float(np.abs(gfd - g[:n_params]).max())}


def bench_c5(fsv, torch, stream, steps=5, warmup=1, packets=False):
    """The 30-qubit workload (14 electrons, 500 operators): FP64 and FP32
    energy + adjoint-gradient rates on the sector engine, the dominant
    kernel's roofline, and finite differences on 16 parameters.  The oracle
    is not run at this size (the 24-qubit cpu_baseline stands)."""
    from workloads import config
    p = config("C5")
    k = p.n_ops
    psi = torch.empty(1 << p.n_qubits, dtype=torch.complex128, device=torch.device("cuda:0"))
    lam = torch.empty_like(psi)
    print(f"[bench] C5 n={p.n_qubits} K={k}: building the plan", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    plan, ms, evals_s, stages, e, g = time_engine(fsv, torch, p, 0, "sector", steps, warmup, stream, psi, lam)
    setup_s = time.perf_counter() - t0
    mb = sector_model_bytes(p, 8)
    start, tiles = plan.runs(adjoint=True)
    fused_runs = len({start[t] for t in range(k) if tiles[t] > 0})
    if fused_runs == 0:
        roof = roofline_of(mb, stages, k, "k_cadj_zip<double> (sector adjoint step on (psi, lam) pairs)",
                           traffic_from_profile("C5", C5_PROFILE, rotation_source_hash))
    else:
        roof = None
    fd = fd_subset(plan, p, g, psi, lam)
    fd["adjoint_speedup_extrapolated"] = fd["extrapolated_full_fd_s"] / (ms * 1e-3)
    print(f"[bench] C5: {ms:.2f} ms/eval; FD on 16 parameters {fd['measured_s']:.2f} s, "
          f"extrapolated {fd['extrapolated_full_fd_s']:.1f} s", file=sys.stderr, flush=True)
    del plan
    p32, ms32, evals32, st32, e32, g32 = time_engine(
        fsv, torch, p, 1, "sector", steps, warmup, stream,
        psi.view(torch.float64)[: psi.numel()].view(torch.complex64),
        lam.view(torch.float64)[: lam.numel()].view(torch.complex64))
    del p32
    pk = None
    if packets:
        # component packets on request (FSV_FUSE=packets at plan creation):
        # every run is a packet run; planning takes minutes at this size
        print("[bench] C5 with packet runs on request: building the plan", file=sys.stderr, flush=True)
        os.environ["FSV_FUSE"] = "packets"
        os.environ["FSV_VERBOSE"] = "1"  # the library prints one line per planned run
        try:
            t0 = time.perf_counter()
            plan_pk = fsv.Plan(p, device=psi.device)
            plan_s = time.perf_counter() - t0
        finally:
            del os.environ["FSV_FUSE"]
            del os.environ["FSV_VERBOSE"]
        for _ in range(warmup):
            plan_pk.energy_grad(p.theta, psi, lam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            e_pk, g_pk = plan_pk.energy_grad(p.theta, psi, lam)
        torch.cuda.synchronize()
        ms_pk = (time.perf_counter() - t0) * 1e3 / steps
        start_pk, tiles_pk = plan_pk.runs(adjoint=True)
        pk = {"plan_creation_s": plan_s, "device_bytes": plan_pk.device_bytes, "ms_per_eval": ms_pk,
              "evals_s": 1e3 / ms_pk, "packet_runs": len({int(start_pk[t]) for t in range(k) if tiles_pk[t] > 0}),
              "abs_energy_diff_vs_default": abs(e_pk - e),
              "max_abs_grad_diff_vs_default": float(np.abs(g_pk - g).max())}
        del plan_pk
        print(f"[bench] C5 packets on request: {ms_pk:.2f} ms/eval, plan {plan_s:.0f} s", file=sys.stderr, flush=True)
    return {"workload": f"C5: {p.n_qubits} qubits, {p.n_alpha + p.n_beta} electrons, {k} sampled "
                        "spin-conserving singles/doubles, energy + adjoint gradient",
            "evals_s": evals_s, "ms_per_eval": ms, "steps": steps, "warmup": warmup, "dtype": "f64",
            "stage_ms": stages, "energy": e, "fused_adjoint_runs": fused_runs,
            "hbm_frac_sector_model": mb["eval"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "roofline": roof,
            "fp32_variant": {"evals_s": evals32, "ms_per_eval": ms32, "stage_ms": st32,
                             "abs_energy_error_vs_fp64_Ha": abs(e32 - e),
                             "max_abs_grad_error_vs_fp64": float(np.abs(g32 - g).max())},
            "fd_subset": fd, "plan_setup_and_timing_s": setup_s, "packets_on_request": pk}


ORACLE_SAMPLE = r"""
import sys, time, json
sys.path.insert(0, sys.argv[1])
from oracle import sector
from workloads import config
p = config(sys.argv[2])
sector.build()
sector.energy_grad(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, p.e_core, p.ordering) if p.n_qubits < 20 else None
t0 = time.perf_counter(); n = 0
while True:
    sector.energy_grad(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, p.e_core, p.ordering)
    n += 1
    el = time.perf_counter() - t0
    if el >= float(sys.argv[3]):
        break
print(json.dumps({"n": n, "s": el, "threads": sector.num_threads()}))
"""


def oracle_sample(name, seconds, threads=None):
    """The oracle's energy + adjoint gradient on config `name`, repeated for
    about `seconds`, in a child process (OMP_NUM_THREADS = threads when
    given)."""
    import subprocess
    env = dict(os.environ)
    if threads:
        env["OMP_NUM_THREADS"] = str(threads)
    r = subprocess.run([sys.executable, "-c", ORACLE_SAMPLE, ROOT, name, str(seconds)], env=env,
                       capture_output=True, text=True, check=True)
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, max_seconds=30.0):
    from oracle import sector
    sector.build()
    t0 = time.perf_counter()
    n = 0
    while True:
        sector.energy_grad(p.n_orb, p.n_alpha, p.n_beta, p.ops, p.theta, p.h, p.g, p.e_core, p.ordering)
        n += 1
        el = time.perf_counter() - t0
        if el >= min(10.0, max_seconds):  # a sample of about 10 s of oracle work
            break
    out = {"value": n / el, "unit": "evals/s", "cores": sector.num_threads(), "kind": "oracle",
           "sample": f"{n} full energy+adjoint-gradient evaluation(s) of the same {p.n_qubits}-qubit workload "
                     f"(sector-compressed FP64 C/OpenMP oracle), {el:.1f} s",
           "cpu_model": cpu_model(), "host_cpus": len(os.sched_getaffinity(0))}
    # the same on one thread, and the small configurations on all threads and on one
    one = oracle_sample("C3", 8.0, threads=1)
    out["single_thread"] = {"value": one["n"] / one["s"], "unit": "evals/s", "cores": one["threads"],
                            "sample": f"{one['n']} evaluation(s) of the {p.n_qubits}-qubit workload, {one['s']:.1f} s"}
    small = {}
    for name in ("C1", "C2"):
        a = oracle_sample(name, 1.0)
        b = oracle_sample(name, 1.0, threads=1)
        small[name] = {"all_threads_evals_s": a["n"] / a["s"], "threads": a["threads"],
                       "single_thread_evals_s": b["n"] / b["s"]}
    out["small_configs"] = small
    return out


def quiet_gc():
    """Collect, then move every live object out of the collector's reach: a
    full collection over torch's objects stalls the host for ~35 ms, which a
    timed loop of ~1 ms steps would otherwise absorb at random."""
    gc.collect()
    gc.freeze()


def time_engine(fsv, torch, p, precision, engine, steps, warmup, stream, psi, lam):
    """Timed energy+gradient passes of one engine, then per-stage HIP-event
    timing on the plan's stream."""
    plan = fsv.Plan(p, precision=precision, device=psi.device, engine=engine)
    quiet_gc()
    for _ in range(warmup):
        plan.energy_grad(p.theta, psi, lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        e, g = plan.energy_grad(p.theta, psi, lam)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t_fwd, t_sig, t_rev = [], [], []
    for _ in range(max(3, min(steps, 10))):
        plan.set_theta(p.theta)
        ev[0].record(stream)
        plan.forward_async(psi)
        ev[1].record(stream)
        plan.sigma_async(psi, lam)
        ev[2].record(stream)
        plan.reverse_async(psi, lam)
        ev[3].record(stream)
        plan.finish()
        torch.cuda.synchronize()
        t_fwd.append(ev[0].elapsed_time(ev[1]))
        t_sig.append(ev[1].elapsed_time(ev[2]))
        t_rev.append(ev[2].elapsed_time(ev[3]))
    stages = {"forward": float(np.median(t_fwd)), "sigma": float(np.median(t_sig)),
              "reverse": float(np.median(t_rev))}
    print(f"[bench] {engine}: {ms:.3f} ms/eval; stages forward {stages['forward']:.3f} ms, "
          f"sigma {stages['sigma']:.3f} ms, reverse {stages['reverse']:.3f} ms",
          file=sys.stderr, flush=True)
    return plan, ms, steps / (t1 - t0), stages, e, g


def roofline_of(mb, stages, k, kernel, traffic=None):
    """Adjoint-step kernel: algorithmic bytes per launch over its average launch
    duration (the reverse stage's HIP-event time over its K launches)."""
    launch_ms = stages["reverse"] / k
    per_launch = mb["reverse"] / k
    achieved = per_launch / (launch_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
            "avg_launch_us": launch_ms * 1e3, "algorithmic_bytes_per_launch": per_launch}


ROTATION_SOURCE = os.path.join(ROOT, "paper_2405_11567_amd", "csrc", "fsv_sigma.hip")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_cadj_zip_sector_24q_fp64.md")
PACKET_SOURCE = os.path.join(ROOT, "paper_2405_11567_amd", "csrc", "fsv_packet.hip")
PACKET_PROFILE = os.path.join(ROOT, "profiles", "k_pkt_adjoint_24q_fp64.md")
C5_PROFILE = os.path.join(ROOT, "profiles", "k_cadj_zip_sector_30q_fp64.md")


def rotation_source_hash():
    """sha256 (16 hex digits) of the rotation-kernel section of the sector
    kernel file: the launch-grid helper, pair decoding, k_crot, k_cadj, k_zip and
    k_cadj_zip."""
    import hashlib
    text = open(ROTATION_SOURCE).read()
    a = text.index("// ------------------------------------------------------------ rotations ----")
    b = text.index("// ---------------------------------------------------------------- sigma ----")
    return hashlib.sha256(text[a:b].encode()).hexdigest()[:16]


def packet_source_hash():
    """sha256 (16 hex digits) of the packet source file: its kernels and the
    host code that forms runs and packs components (both set the traffic)."""
    import hashlib
    return hashlib.sha256(open(PACKET_SOURCE, "rb").read()).hexdigest()[:16]


def traffic_from_profile(workload, path=TRAFFIC_PROFILE, source_hash=rotation_source_hash):
    """HBM bytes per launch of a profiled kernel from its committed rocprofv3
    counter summary (FETCH_SIZE x calibration + WRITE_SIZE), when it was taken
    on the current kernel source and this workload; otherwise None."""
    try:
        fields = {}
        for line in open(path):
            if ":" in line and line.startswith("- "):
                key, val = line[2:].split(":", 1)
                fields[key.strip()] = val.strip().strip("`")
        if fields.get("source_sha256") != source_hash() or fields.get("workload") != workload:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def sector_strings(m, n):
    from itertools import combinations
    return np.array(sorted(sum(1 << b for b in c) for c in combinations(range(m), n)), dtype=np.int64)


def run_touched(p, k0, k1):
    """Sector amplitudes (alpha string rank * n_beta_strings + beta rank) that
    the operators k0..k1-1 pair: the amplitudes a fused run must move."""
    m, na, nb = p.n_orb, p.n_alpha, p.n_beta
    sa, sb = sector_strings(m, na), sector_strings(m, nb)
    rank = {0: np.full(1 << m, -1, np.int64), 1: np.full(1 << m, -1, np.int64)}
    rank[0][sa] = np.arange(len(sa))
    rank[1][sb] = np.arange(len(sb))
    strs = {0: sa, 1: sb}
    out = []
    for op in p.ops[k0:k1]:
        a, b, j, i = (int(v) for v in op)
        ends = []
        for sp in (0, 1):
            ann = sum(1 << (v // 2) for v in (i, j) if v >= 0 and v % 2 == sp)
            cre = sum(1 << (v // 2) for v in (a, b) if v >= 0 and v % 2 == sp)
            S = strs[sp]
            if not ann and not cre:
                ends.append((np.arange(len(S)), np.arange(len(S))))
                continue
            src = S[((S & ann) == ann) & ((S & (cre & ~ann)) == 0)]
            ends.append((rank[sp][src], rank[sp][(src & ~ann) | cre]))
        nsb = len(sb)
        for t in (0, 1):
            out.append((ends[0][t][:, None] * nsb + ends[1][t][None, :]).ravel())
    return int(len(np.unique(np.concatenate(out)))) if out else 0


def packet_roofline(fsv, torch, plan, p, precision, psi, lam, traffic=None, reps=5):
    """Roofline of the adjoint packet-run kernel: the adjoint sweep is launched
    eagerly and each packet kernel's own start and end go to HIP events
    (fsv_time_runs); achieved = algorithmic bytes of the packet runs (their
    touched amplitudes, psi and lam, read and written) over their measured
    time.  None when the plan has no packet runs."""
    start, tiles = plan.runs(adjoint=True)
    k = len(start)
    firsts = [t for t in range(k) if t == 0 or start[t] != start[t - 1]]
    groups = [(k0, (firsts[n + 1] if n + 1 < len(firsts) else k)) for n, k0 in enumerate(firsts)]
    fused = [n for n, (k0, k1) in enumerate(groups) if tiles[k0] > 0]
    if not fused:
        return None
    times = []
    for _ in range(reps + 1):
        plan.set_theta(p.theta)
        plan.forward_async(psi)
        plan.sigma_async(psi, lam)
        times.append(plan.time_runs(psi, lam, adjoint=True))
        torch.cuda.synchronize()
    med = np.median(np.array(times[1:]), axis=0)
    es = 8 if precision == 0 else 4
    amps = [run_touched(p, *groups[n]) for n in fused]
    byts = [4.0 * es * a for a in amps]  # psi and lam, read and written
    ms = [float(med[n]) for n in fused]
    achieved = sum(byts) / (sum(ms) * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_pkt<%s, true> (adjoint packet run)" % ("double" if precision == 0 else "float"),
            "avg_launch_us": float(np.mean(ms)) * 1e3,
            "algorithmic_bytes_per_launch": float(np.mean(byts)),
            "launches_per_eval": len(fused),
            "operators_fused": int(sum(groups[n][1] - groups[n][0] for n in fused)),
            "mean_touched_amplitudes": float(np.mean(amps)),
            "mean_packets": float(np.mean([tiles[groups[n][0]] for n in fused])),
            "adjoint_sweep_ms": float(med.sum())}


def unfused_reverse(fsv, torch, p, precision, stream, psi, lam, reps=5):
    """Reverse-stage HIP-event time of a plan without fused runs: K launches of
    the per-operator adjoint kernel."""
    os.environ["FSV_NO_FUSE"] = "1"
    try:
        plan = fsv.Plan(p, precision=precision, device=psi.device)
    finally:
        os.environ.pop("FSV_NO_FUSE", None)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    times = []
    for _ in range(reps + 1):
        plan.set_theta(p.theta)
        plan.forward_async(psi)
        plan.sigma_async(psi, lam)
        ev[0].record(stream)
        plan.reverse_async(psi, lam)
        ev[1].record(stream)
        plan.finish()
        torch.cuda.synchronize()
        times.append(ev[0].elapsed_time(ev[1]))
    return float(np.median(times[1:]))


def bench_pool(fsv, torch, p, psi, lam, stages, reps=10):
    """ADAPT screening of the whole UCCSD pool at psi(theta): forward sweep,
    H psi, and every pool operator's 2 Re<H psi|T|psi> in one launch;
    fermionic and qubit-excitation pools."""
    from workloads import uccsd_pool
    pool_ops = np.asarray(uccsd_pool(p.n_orb, p.n_alpha, p.n_beta), dtype=np.int32)
    plan = fsv.Plan(p, device=psi.device)
    quiet_gc()
    from math import comb
    m, na, nb = p.n_orb, p.n_alpha, p.n_beta
    pair_bytes = sum(4 * 8 * sector_pairs(op, m, na, nb) for op in pool_ops)  # read psi, lam at both ends
    out = {"pool_ops": int(len(pool_ops))}
    for exc, name in ((0, "fermionic"), (1, "qubit")):
        pool = plan.pool(pool_ops, excitation=exc)
        pool.gradients(p.theta, psi, lam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            e, g = pool.gradients(p.theta, psi, lam)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        screen_ms = max(ms - stages["forward"] - stages["sigma"], 1e-6)
        out[name] = {"ms_per_screening": ms, "screen_ms_beyond_state": screen_ms,
                     "pool_gradients_per_s": len(pool_ops) / (ms * 1e-3),
                     "screen_algorithmic_GBs": pair_bytes / (screen_ms * 1e-3) / 1e9,
                     "max_abs_grad": float(np.abs(g).max())}
        print(f"[bench] {name} pool of {len(pool_ops)}: {ms:.3f} ms per screening", file=sys.stderr, flush=True)
        pool.close()
    plan.close()
    return out


def bench_multidet(fsv, torch, p, psi, lam, n_det=10000, reps=10):
    """Energy + gradient from a 10^4-determinant start (the size of the
    paper's warm starts), and a one-body property (tr(d gamma)) of psi."""
    rng = np.random.default_rng(2024)
    m, na, nb = p.n_orb, p.n_alpha, p.n_beta
    # random distinct sector determinants as qubit strings: random alpha and
    # beta occupations in the plan's ordering
    def qubit(so):
        pp, sp = divmod(so, 2)
        return so if p.ordering == 0 else pp + sp * m
    seen, dets = set(), []
    while len(dets) < n_det:
        a = rng.choice(m, na, replace=False)
        b = rng.choice(m, nb, replace=False)
        x = 0
        for q in a:
            x |= 1 << qubit(2 * int(q))
        for q in b:
            x |= 1 << qubit(2 * int(q) + 1)
        if x not in seen:
            seen.add(x)
            dets.append(x)
    coef = rng.normal(size=n_det)
    coef /= np.linalg.norm(coef)
    plan = fsv.Plan(p, device=psi.device)
    plan.set_initial_state(np.array(dets, dtype=np.uint64), coef)
    quiet_gc()
    plan.energy_grad(p.theta, psi, lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        e, _ = plan.energy_grad(p.theta, psi, lam)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    plan.ansatz_apply(p.theta, psi)
    d = rng.normal(size=(m, m))
    d = d + d.T
    t1 = time.perf_counter()
    val = plan.onebody_expectation(psi, d)
    prop_ms = (time.perf_counter() - t1) * 1e3
    plan.close()
    print(f"[bench] {n_det}-determinant start: {ms:.3f} ms per energy+gradient", file=sys.stderr, flush=True)
    return {"n_det": n_det, "ms_per_eval": ms, "evals_s": 1e3 / ms, "energy": e,
            "onebody_property_ms": prop_ms, "onebody_property": val.real}


def bench_strategy2(fsv, torch, p, psi, lam, outer=10, inner=5, kappa=0.0, reps=5):
    """The 24-qubit workload's self-consistent loop (Strategy 2): per outer
    iteration set the one-body potential, five gradient-descent steps on the
    angles (energy + adjoint gradient, theta -= 0.1 grad), then the ansatz
    state, its energy and its 1-RDM, from which the next potential is built
    (10 outer iterations; the stand-in functional with kappa = 0, so the
    potential is the fixed v0).  Reports the first outer iteration whose
    energy change is below 1e-4 Ha, and each call of the loop timed on its
    own."""
    from paper_2405_11567_amd.scloop import self_consistent_loop
    from workloads import potential_v0
    plan = fsv.Plan(p, device=psi.device)
    v0 = potential_v0(p.n_orb)
    self_consistent_loop(plan, p.theta, v0, p.n_alpha, p.n_beta, kappa=kappa, outer=1, inner=1, lr=0.1,
                         psi=psi, lam=lam)
    quiet_gc()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = self_consistent_loop(plan, p.theta, v0, p.n_alpha, p.n_beta, kappa=kappa, outer=outer, inner=inner,
                               lr=0.1, threshold=1e-4, psi=psi, lam=lam)
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - t0) * 1e3

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / reps

    plan.ansatz_apply(p.theta, psi)
    out = {"outer_iterations": outer, "inner_steps": inner, "kappa": kappa, "threshold_Ha": 1e-4,
           "energies": [r.energy for r in res.records], "delta_E": [None if np.isnan(r.delta) else r.delta for r in res.records],
           "loop_ms": loop_ms, "ms_per_outer_iteration": loop_ms / outer,
           "rdm1_ms": timed(lambda: plan.rdm1(psi)),
           "set_onebody_potential_ms": timed(lambda: plan.set_onebody_potential(v0)),
           "ansatz_apply_ms": timed(lambda: plan.ansatz_apply(p.theta, psi)),
           "energy_ms": timed(lambda: plan.energy(psi)),
           "first_converged_iteration": res.first_converged,
           "last_energy": res.records[-1].energy, "last_e2": res.records[-1].e2}
    plan.set_onebody_potential(None)
    print(f"[bench] strategy-2 loop: {outer} outer iterations in {loop_ms:.2f} ms; 1-RDM {out['rdm1_ms']:.3f} ms",
          file=sys.stderr, flush=True)
    return out


def run_batch(steps, warmup, tune=False, fd=True):
    """C4: 256 independent instances (10..20 qubits), energy + adjoint gradient
    of every instance per step in one graph launch; compared with one plan
    per instance called in a loop, and with the finite-difference gradient
    of every instance (each plan's own 2K + 1 energies)."""
    import torch
    import paper_2405_11567_amd as fsv
    from workloads import batch_config

    probs = batch_config()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    b = fsv.Batch(probs, device=dev)
    # all angles as one flat array (the batch's own layout), so that a step
    # times the library call and not per-instance array marshalling
    thetas = np.concatenate([p.theta for p in probs])
    tune_report = b.autotune() if tune else ""
    if tune_report:
        print(tune_report, file=sys.stderr, flush=True)
    quiet_gc()
    for _ in range(warmup):
        b.energy_grad(thetas)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        e, g = b.energy_grad(thetas)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    print(f"[bench] batch of {len(probs)}: {dt*1e3:.3f} ms per step", file=sys.stderr, flush=True)
    # unbatched: one plan per instance, sector engine, called in sequence
    plans = [fsv.Plan(p, device=dev) for p in probs]
    bufs = [(pl.new_state(), pl.new_state()) for pl in plans]
    for pl, p, (ps, lm) in zip(plans, probs, bufs):
        pl.energy_grad(p.theta, ps, lm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    worst = 0.0
    for i, (pl, p, (ps, lm)) in enumerate(zip(plans, probs, bufs)):
        eu, gu = pl.energy_grad(p.theta, ps, lm)
        worst = max(worst, abs(eu - e[i]))
    torch.cuda.synchronize()
    du = time.perf_counter() - t1
    print(f"[bench] unbatched loop: {du*1e3:.3f} ms", file=sys.stderr, flush=True)
    fd_out = None
    if fd:
        t2 = time.perf_counter()
        worst_fd = 0.0
        off = 0
        for pl, p, (ps, lm) in zip(plans, probs, bufs):
            _, gfd = pl.energy_grad_fd(p.theta, 1e-5, ps)
            worst_fd = max(worst_fd, float(np.abs(gfd - g[off:off + p.n_ops]).max()))
            off += p.n_ops
        torch.cuda.synchronize()
        dfd = time.perf_counter() - t2
        fd_out = {"s": dfd, "energies": int(sum(2 * p.n_ops + 1 for p in probs)), "batch_speedup": dfd / dt,
                  "max_abs_diff_vs_batch_gradient": worst_fd}
        print(f"[bench] finite differences, every instance: {dfd:.3f} s", file=sys.stderr, flush=True)
    return {
        "workload": "C4: 256 instances, qubits uniform in 10..20 (even), electrons n/2 +- 2, 50..150 "
                    "operators each, energy + adjoint gradient",
        "instances": len(probs), "total_ops": int(sum(p.n_ops for p in probs)),
        "instance_evals_s": len(probs) / dt, "ms_per_step": dt * 1e3, "steps": steps, "warmup": warmup,
        "unbatched": {"ms": du * 1e3, "instance_evals_s": len(probs) / du,
                      "batch_speedup": du / dt, "max_abs_dE_vs_batch": worst},
        "fd_every_instance": fd_out,
        "batch_device_bytes": b.bytes,
    }


def bench_batch(args):
    r = run_batch(args.steps, args.warmup, args.tune)
    out = {
        "metric": "batched energy+gradient instance-evals/s (256 instances, 10-20 qubits)",
        "value": r["instance_evals_s"], "unit": "instance-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": r["workload"], "instances": r["instances"], "total_ops": r["total_ops"]},
        "unbatched": r["unbatched"], "fd_every_instance": r["fd_every_instance"],
        "batch_device_bytes": r["batch_device_bytes"],
    }
    print(json.dumps(out))


def bench_small(fsv, torch, reps=60):
    """C1 (energy only: the forward sweep and <H>, through the stage calls)
    and C2 (energy + adjoint gradient, FP64, and the FP32 variant's energy
    error): absolute rates, median and fastest of `reps` timed calls each.
    Both states are cache-resident, so no HBM fraction is given."""
    from workloads import config

    def timed(fn):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts)) * 1e3, float(np.min(ts)) * 1e3

    out = {}
    p1 = config("C1")
    plan = fsv.Plan(p1)
    psi, lam = plan.new_state(), plan.new_state()

    def energy_only():
        plan.set_theta(p1.theta)
        plan.forward_async(psi)
        plan.sigma_async(psi, lam)
        return plan.finish()[0]

    med, mn = timed(energy_only)
    out["C1"] = {"work": "energy only (forward sweep and <H>)", "evals_s": 1e3 / med, "median_ms": med,
                 "min_ms": mn, "energy": energy_only()}
    p2 = config("C2")
    plan = fsv.Plan(p2)
    psi, lam = plan.new_state(), plan.new_state()
    med, mn = timed(lambda: plan.energy_grad(p2.theta, psi, lam))
    e64, _ = plan.energy_grad(p2.theta, psi, lam)
    p32 = fsv.Plan(p2, precision=1)
    e32, _ = p32.energy_grad(p2.theta)
    out["C2"] = {"work": "energy + adjoint gradient", "evals_s": 1e3 / med, "median_ms": med, "min_ms": mn,
                 "energy": e64, "fp32_abs_energy_error_vs_fp64_Ha": abs(e32 - e64)}
    print(f"[bench] C1 energy {out['C1']['median_ms']:.3f} ms, C2 energy+gradient {med:.3f} ms",
          file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C3")
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--engine", default="sector", choices=["sector", "dense"])
    ap.add_argument("--no-dense", action="store_true", help="skip the dense-engine comparison run")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fd", action="store_true")
    ap.add_argument("--no-pool", action="store_true", help="skip the ADAPT pool-screening measurement")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-amplitude variant")
    ap.add_argument("--no-scf", action="store_true", help="skip the Strategy-2 self-consistent loop")
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the legs of the default run beyond the 24-qubit workload (C1, C2, C4, C5)")
    ap.add_argument("--c5-packets", action="store_true",
                    help="also time the 30-qubit workload with component packets on request (minutes of planning)")
    ap.add_argument("--tune", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy three times (the known-size "
                         "reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the state-vector path here is single-GPU "
              "(sharding across GPUs is a design note, not built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.config == "C4":
        return bench_batch(args)

    import torch
    import paper_2405_11567_amd as fsv
    from workloads import config

    p = config(args.config)
    amp_bytes = 16 if args.precision == 0 else 8
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    if args.calibrate_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    dtype = torch.complex128 if args.precision == 0 else torch.complex64
    psi = torch.empty(1 << p.n_qubits, dtype=dtype, device=dev)
    lam = torch.empty_like(psi)
    k = p.n_ops
    print(f"[bench] {args.config} n={p.n_qubits} K={k} precision={args.precision}", file=sys.stderr, flush=True)

    plan, ms, evals_s, stages, e, g = time_engine(fsv, torch, p, args.precision, args.engine,
                                                  args.steps, args.warmup, stream, psi, lam)
    if args.tune:
        print(plan.autotune(psi, lam), file=sys.stderr, flush=True)
    mb_dense = model_bytes(p, amp_bytes)
    # the sector engine stores the (exactly real) state as real FP64 / FP32
    mb_sector = sector_model_bytes(p, amp_bytes // 2)
    mb = mb_sector if args.engine == "sector" else mb_dense
    per_op = None
    if args.engine == "sector":
        rev_ms = unfused_reverse(fsv, torch, p, args.precision, stream, psi, lam)
        print(f"[bench] per-operator adjoint sweep (no fused runs): {rev_ms:.3f} ms", file=sys.stderr, flush=True)
        traffic = traffic_from_profile(args.config) if args.precision == 0 else None
        per_op = roofline_of(mb, {"reverse": rev_ms}, k, "k_cadj_zip<double> (sector adjoint step on (psi, lam) pairs)"
                             if args.precision == 0 else "k_cadj_zip<float> (sector adjoint step on (psi, lam) pairs)",
                             traffic)
        pk_traffic = (traffic_from_profile(args.config, PACKET_PROFILE, packet_source_hash)
                      if args.precision == 0 else None)
        roof = packet_roofline(fsv, torch, plan, p, args.precision, psi, lam, pk_traffic)
        if roof is None:
            roof, per_op = per_op, None
        else:
            print(f"[bench] adjoint packet runs: {roof['launches_per_eval']} launches, "
                  f"{roof['avg_launch_us']:.1f} us each, {roof['achieved']:.0f} GB/s algorithmic",
                  file=sys.stderr, flush=True)
    else:
        roof = roofline_of(mb, stages, k, "k_adj (dense adjoint step)")

    dense = None
    if args.engine == "sector" and not args.no_dense:
        dplan, dms, devals, dstages, de, dg = time_engine(fsv, torch, p, args.precision, "dense",
                                                          max(3, min(args.steps // 3, 20)), 1, stream, psi, lam)
        dense = {"evals_s": devals, "ms_per_eval": dms, "stage_ms": dstages,
                 "roofline": roofline_of(mb_dense, dstages, k, "k_adj (dense adjoint step)"),
                 "dense_model_hbm_frac": mb_dense["eval"] / (dms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "max_abs_dE_vs_sector": abs(de - e), "max_abs_dg_vs_sector": float(np.abs(dg - g).max())}
        del dplan

    fd = None
    if not args.no_fd:
        t2 = time.perf_counter()
        _, gfd = plan.energy_grad_fd(p.theta, 1e-5, psi)
        fd_s = time.perf_counter() - t2
        fd = {"gradient_s": fd_s, "energies": 2 * k + 1, "adjoint_speedup": fd_s / (ms * 1e-3),
              "max_abs_diff_vs_adjoint": float(np.abs(gfd - g).max())}
        print(f"[bench] FD gradient {fd_s:.3f} s ({2*k+1} energies), adjoint {ms:.3f} ms: "
              f"{fd['adjoint_speedup']:.0f}x", file=sys.stderr, flush=True)

    fp32 = None
    if args.precision == 0 and not args.no_fp32:
        # the FP32-amplitude variant on the same workload, its energy error
        # against the FP64 result (which matches the FP64 oracle to 1e-10 Ha)
        p32, ms32, evals32, st32, e32, g32 = time_engine(fsv, torch, p, 1, args.engine, max(3, args.steps // 3), 1,
                                                         stream, psi.view(torch.float64)[: psi.numel()].view(torch.complex64),
                                                         lam.view(torch.float64)[: lam.numel()].view(torch.complex64))
        fp32 = {"evals_s": evals32, "ms_per_eval": ms32, "stage_ms": st32, "energy": e32,
                "abs_energy_error_vs_fp64_Ha": abs(e32 - e), "max_abs_grad_error_vs_fp64": float(np.abs(g32 - g).max())}
        del p32

    pool = None
    if args.engine == "sector" and args.precision == 0 and not args.no_pool:
        pool = bench_pool(fsv, torch, p, psi, lam, stages)
        if fd is not None:
            # screening by finite differences: two energies of the ansatz with
            # each pool operator appended at +-h
            e_ms = fd["gradient_s"] / fd["energies"] * 1e3
            pool["fd_screening_s_estimate"] = 2 * pool["pool_ops"] * e_ms / 1e3

    multidet = None
    if args.engine == "sector" and args.precision == 0 and not args.no_pool:
        multidet = bench_multidet(fsv, torch, p, psi, lam)

    strategy2 = None
    if args.engine == "sector" and args.precision == 0 and not args.no_scf:
        strategy2 = bench_strategy2(fsv, torch, p, psi, lam)

    cpu = None if args.no_cpu else cpu_baseline(p)
    small = c4 = c5 = None
    if args.config == "C3" and args.precision == 0 and args.engine == "sector" and not args.no_c5:
        del plan
        small = bench_small(fsv, torch)
        c4 = run_batch(50, 5)
        c5 = bench_c5(fsv, torch, stream, packets=args.c5_packets)
    out = {
        "metric": f"energy+gradient evals/s and achieved HBM GB/s at {p.n_qubits} qubits vs plain FD method",
        "value": evals_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # the sector engine keeps the exactly real state as real numbers
        "dtype": ({"sector": "f64", "dense": "c128"} if args.precision == 0
                  else {"sector": "f32", "dense": "c64"})[args.engine],
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {p.n_qubits} qubits, {p.n_alpha + p.n_beta} electrons, "
                               f"{k} sampled spin-conserving singles/doubles, energy + adjoint gradient",
                   "n_qubits": p.n_qubits, "n_ops": k, "precision": args.precision,
                   "engine": args.engine},
        "roofline": roof,
        "per_operator_kernel": per_op,
        "eval_model": {"engine_bytes_per_eval": mb["eval"], "stage_ms": stages,
                       "dense_line_model_bytes_per_eval": mb_dense["eval"],
                       "dense_model_hbm_frac": mb_dense["eval"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "dense_engine": dense,
        "energy": e,
        "fd_baseline": fd,
        "fp32_variant": fp32,
        "adapt_pool_screening": pool,
        "multideterminant_start": multidet,
        "strategy2_loop": strategy2,
        "cpu_baseline": cpu,
        "small_configs": small,
        "c4": c4,
        "c5": c5,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
