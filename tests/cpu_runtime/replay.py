"""Replays, on the CPU, the C-ABI call sequences that the GPU tests make, on
the host-check build of the library (libfsv_hostcheck.so: host code under
AddressSanitizer / UndefinedBehaviorSanitizer, HIP replaced by the checking
stand-in of hip_stub.cpp).  Kernels do not run, so no result is checked here:
what is checked is that the host side (table building, packet planning,
graph capture and replay, pinned-buffer copies, the lifetimes of plans,
pools and batches) stays inside its memory and uses only live handles.

Run it with the AddressSanitizer runtime preloaded (see
tests/test_host_replay_cpu.py):  python replay.py <suite>
"""

from __future__ import annotations

import ctypes
import gc
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2405_11567_amd._lib import Problem as CProblem  # noqa: E402
from workloads import batch_config, config, potential_v0, random_problem, uccsd_pool  # noqa: E402

BUILD = os.path.join(HERE, "_build")
stub = ctypes.CDLL(os.path.join(BUILD, "libhipstub.so"), mode=ctypes.RTLD_GLOBAL)
lib = ctypes.CDLL(os.path.join(BUILD, "libfsv_hostcheck.so"))

vp = ctypes.c_void_p
D = ctypes.POINTER(ctypes.c_double)
I32 = ctypes.POINTER(ctypes.c_int32)
stub.hipMalloc.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t]
stub.hipFree.argtypes = [vp]
stub.hip_stub_launches.restype = ctypes.c_ulong
stub.hip_stub_replays.restype = ctypes.c_ulong
stub.hip_stub_live_device_bytes.restype = ctypes.c_size_t
stub.hip_stub_live_handles.restype = ctypes.c_size_t
lib.fsv_last_error.restype = ctypes.c_char_p
for name, args in {
    "fsv_plan_create": [ctypes.POINTER(vp), ctypes.POINTER(CProblem), vp],
    "fsv_plan_destroy": [vp], "fsv_plan_set_engine": [vp, ctypes.c_int],
    "fsv_plan_runs": [vp, ctypes.c_int, I32, I32],
    "fsv_time_runs": [vp, ctypes.c_int, vp, vp, ctypes.POINTER(ctypes.c_float)],
    "ansatz_apply": [vp, D, vp], "energy": [vp, vp, D], "energy_grad": [vp, D, vp, vp, D, D],
    "energy_grad_noalloc": [vp, D, vp, vp, D, D],
    "energy_grad_fd": [vp, D, ctypes.c_double, vp, D, D], "rdm1": [vp, vp, D],
    "set_onebody_potential": [vp, D], "fsv_set_theta": [vp, D], "fsv_forward_async": [vp, vp],
    "fsv_sigma_async": [vp, vp, vp], "fsv_reverse_async": [vp, vp, vp], "fsv_finish": [vp, D, D],
    "fsv_autotune": [vp, vp, vp, ctypes.POINTER(ctypes.c_char_p)],
    "fsv_pool_create": [ctypes.POINTER(vp), vp, I32, ctypes.c_int32, ctypes.c_int32],
    "fsv_pool_destroy": [vp], "fsv_pool_gradients": [vp, D, vp, vp, D, D],
    "fsv_set_initial_state": [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64), D],
    "onebody_expectation": [vp, vp, D, D],
    "fsv_batch_create": [ctypes.POINTER(vp), ctypes.POINTER(CProblem), ctypes.c_int32, vp],
    "fsv_batch_destroy": [vp], "fsv_batch_energy_grad": [vp, D, vp, D, D],
    "fsv_batch_autotune": [vp, vp, ctypes.POINTER(ctypes.c_char_p)],
}.items():
    getattr(lib, name).argtypes = args
    getattr(lib, name).restype = ctypes.c_int
for name in ("fsv_state_bytes", "fsv_plan_workspace_bytes", "fsv_plan_device_bytes", "fsv_batch_arena_bytes",
             "fsv_batch_bytes"):
    getattr(lib, name).restype = ctypes.c_size_t
    getattr(lib, name).argtypes = [vp]
lib.fsv_plan_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
lib.fsv_plan_set_workspace.restype = ctypes.c_int


def dp(a):
    return a.ctypes.data_as(D)


def ok(rc, what):
    if rc < 0:
        raise RuntimeError(f"{what}: {rc} {lib.fsv_last_error().decode()}")
    return rc


class Dev:
    """A device buffer of the stand-in runtime."""

    def __init__(self, nbytes):
        self.p = vp()
        ok(stub.hipMalloc(ctypes.byref(self.p), nbytes), "hipMalloc")

    def free(self):
        if self.p:
            stub.hipFree(self.p)
            self.p = vp()


def cproblem(p, precision=0, keep=None):
    h = np.ascontiguousarray(p.h, dtype=np.float64)
    g = np.ascontiguousarray(p.g, dtype=np.float64)
    ops = np.ascontiguousarray(np.asarray(p.ops, dtype=np.int32).reshape(-1, 4))
    keep.extend([h, g, ops])
    return CProblem(p.n_qubits, p.n_alpha, p.n_beta, p.ordering, precision, dp(h), dp(g),
                    float(getattr(p, "e_core", 0.0)), ops.shape[0], ops.ctypes.data_as(I32),
                    int(getattr(p, "excitation", 0)))


def make_plan(p, precision=0, engine=0):
    keep = []
    cp = cproblem(p, precision, keep)
    h = vp()
    ok(lib.fsv_plan_create(ctypes.byref(h), ctypes.byref(cp), None), "plan_create")
    if engine:
        ok(lib.fsv_plan_set_engine(h, engine), "set_engine")
    return h


def exercise_plan(p, precision=0, engine=0, fd=False, stages=True, extras=True, caller_ws=None):
    """The calls a GPU parity test makes on one plan.  The device memory the
    plan reports owning must be exactly what it allocated: its tables after
    creation, plus its own workspace once a call needed one, or the tables
    alone with a caller workspace (every other case a caller workspace)."""
    live0 = stub.hip_stub_live_device_bytes()
    plan = make_plan(p, precision, engine)
    tables = lib.fsv_plan_device_bytes(plan)
    if stub.hip_stub_live_device_bytes() - live0 != tables:
        raise RuntimeError("fsv_plan_device_bytes does not match the plan's allocations")
    global _ws_turn
    _ws_turn = (_ws_turn + 1) % 2
    wsb = lib.fsv_plan_workspace_bytes(plan)
    ws = None
    if caller_ws if caller_ws is not None else _ws_turn:
        ws = Dev(wsb)
        ok(lib.fsv_plan_set_workspace(plan, ws.p, wsb), "set_workspace")
        if lib.fsv_plan_set_workspace(plan, ws.p, wsb - 8) != -1:
            raise RuntimeError("a too-small workspace must be rejected")
    k = p.n_ops
    sb = lib.fsv_state_bytes(plan)
    psi, lam = Dev(sb), Dev(sb)
    th = np.ascontiguousarray(p.theta, dtype=np.float64)
    e = ctypes.c_double()
    grad = np.zeros(max(k, 1))
    for _ in range(2):  # capture, then replay
        ok(lib.energy_grad(plan, dp(th), psi.p, lam.p, ctypes.byref(e), dp(grad)), "energy_grad")
    psi2, lam2 = Dev(sb), Dev(sb)  # new buffers: the graph is captured again
    ok(lib.energy_grad(plan, dp(th), psi2.p, lam2.p, ctypes.byref(e), dp(grad)), "energy_grad")
    rc = lib.energy_grad_noalloc(plan, dp(th), psi.p, lam.p, ctypes.byref(e), dp(grad))
    if rc not in ((0, -1) if engine == 0 else (-4,)):
        raise RuntimeError(f"energy_grad_noalloc: {rc} {lib.fsv_last_error().decode()}")
    own = lib.fsv_plan_device_bytes(plan) - tables
    if own != (0 if ws else wsb):
        raise RuntimeError(f"plan-owned workspace {own} bytes, expected {0 if ws else wsb}")
    ok(lib.ansatz_apply(plan, dp(th), psi.p), "ansatz_apply")
    ok(lib.energy(plan, psi.p, ctypes.byref(e)), "energy")
    if extras:
        m = p.n_qubits // 2
        gam = np.zeros(4 * m * m)
        ok(lib.rdm1(plan, psi.p, dp(gam)), "rdm1")
        v = np.ascontiguousarray(potential_v0(m, seed=12))
        ok(lib.set_onebody_potential(plan, dp(v)), "potential")
        ok(lib.energy_grad(plan, dp(th), psi.p, lam.p, ctypes.byref(e), dp(grad)), "energy_grad")
        ok(lib.set_onebody_potential(plan, None), "potential")
        d = np.ascontiguousarray(np.arange(m * m, dtype=np.float64).reshape(m, m))
        out = np.zeros(2)
        ok(lib.onebody_expectation(plan, psi.p, dp(d), dp(out)), "onebody_expectation")
    if stages:
        for _ in range(2):
            ok(lib.fsv_set_theta(plan, dp(th)), "set_theta")
            ok(lib.fsv_forward_async(plan, psi.p), "forward")
            ok(lib.fsv_sigma_async(plan, psi.p, lam.p), "sigma")
            ok(lib.fsv_reverse_async(plan, psi.p, lam.p), "reverse")
            ok(lib.fsv_finish(plan, ctypes.byref(e), dp(grad)), "finish")
    if fd:
        ok(lib.energy_grad_fd(plan, dp(th), 1e-5, psi.p, ctypes.byref(e), dp(grad)), "fd")
    for b in (psi, lam, psi2, lam2):
        b.free()
    ok(lib.fsv_plan_destroy(plan), "destroy")
    if ws:
        ws.free()
    if stub.hip_stub_live_device_bytes() != live0:
        raise RuntimeError("the plan left device memory behind")


_ws_turn = 0


def with_env(env, fn):
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        fn()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def sigma_problem(nfac):
    p = random_problem(14, 7, 40, seed=600 + nfac, theta_std=0.3, replace=True)
    m = p.n_orb
    rng = np.random.default_rng(nfac)
    g = np.zeros((m, m, m, m))
    for _ in range(nfac):
        l = rng.normal(0, 0.05, (m, m))
        l = l + l.T
        g += np.einsum("pq,rs->pqrs", l, l)
    p.g = g
    return p


def suite_sigma():
    for nfac in (8, 12, 40):
        for mode in ("direct", "lowrank", "auto"):
            p = sigma_problem(nfac)
            print("sigma paths", nfac, mode, flush=True)
            for engine in (0, 1):
                with_env({"FSV_SIGMA": mode}, lambda: exercise_plan(p, engine=engine))


def suite_parity():
    for ordering in (0, 1):
        for precision in (0, 1):
            for engine in (0, 1):
                exercise_plan(config("C1", ordering), precision, engine, fd=True)
    for (n, ne, k, seed, ordering) in [(10, 5, 40, 201, 0), (12, 6, 60, 202, 1), (14, 7, 80, 203, 0),
                                       (16, 8, 60, 204, 1), (16, 5, 50, 205, 0), (18, 9, 40, 206, 1)]:
        p = random_problem(n, ne, k, seed=seed, theta_std=0.6, replace=True, ordering=ordering)
        print("random", n, ne, k, flush=True)
        for engine in (0, 1):
            exercise_plan(p, engine=engine, extras=False, stages=False)
    for ordering in (0, 1):
        for engine in (0, 1):
            print("C2", ordering, engine, flush=True)
            exercise_plan(config("C2", ordering), engine=engine)
    for (n, ne, k) in [(8, 4, 0), (10, 1, 5), (8, 8, 0), (2, 1, 0), (4, 2, 3), (8, 7, 6)]:
        p = random_problem(n, ne, k if k else None, seed=500 + n + ne, theta_std=0.3, replace=True)
        if k == 0:
            p.ops = np.zeros((0, 4), dtype=np.int32)
            p.theta = np.zeros(0)
        print("edge", n, ne, k, flush=True)
        for engine in (0, 1):
            exercise_plan(p, engine=engine)
    p = random_problem(16, 8, 120, seed=801, theta_std=0.5, replace=True, ordering=1)
    for env in ({}, {"FSV_NO_FUSE": "1"}, {"FSV_FORCE_FUSE": "1"}, {"FSV_FUSE": "tiles"}, {"FSV_FUSE": "packets"}):
        for precision in (0, 1):
            print("fused", env, precision, flush=True)
            with_env(env, lambda: exercise_plan(p, precision))
    for same_spin in ("dense", "sparse"):
        for split in ("", "1"):
            env = {"FSV_SAME_SPIN": same_spin}
            if split:
                env["FSV_LR_SPLIT"] = split
            print("same-spin", env, flush=True)
            for engine in (0, 1):
                with_env(env, lambda: exercise_plan(config("C2", 1), engine=engine))
    # autotune and per-run timing
    p = config("C2")
    plan = make_plan(p)
    sb = lib.fsv_state_bytes(plan)
    psi, lam = Dev(sb), Dev(sb)
    rep = ctypes.c_char_p()
    ok(lib.fsv_autotune(plan, psi.p, lam.p, ctypes.byref(rep)), "autotune")
    th = np.ascontiguousarray(p.theta)
    e = ctypes.c_double()
    grad = np.zeros(p.n_ops)
    ok(lib.energy_grad(plan, dp(th), psi.p, lam.p, ctypes.byref(e), dp(grad)), "energy_grad")
    nruns = ok(lib.fsv_plan_runs(plan, 0, None, None), "runs")
    ms = np.zeros(max(nruns, 1), dtype=np.float32)
    ok(lib.fsv_time_runs(plan, 0, psi.p, None, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), "time")
    nruns = ok(lib.fsv_plan_runs(plan, 1, None, None), "runs")
    ms = np.zeros(max(nruns, 1), dtype=np.float32)
    ok(lib.fsv_time_runs(plan, 1, psi.p, lam.p, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), "time")
    psi.free()
    lam.free()
    ok(lib.fsv_plan_destroy(plan), "destroy")


def suite_pools():
    for ordering in (0, 1):
        p = config("C2", ordering)
        plan = make_plan(p)
        sb = lib.fsv_state_bytes(plan)
        psi, lam = Dev(sb), Dev(sb)
        pool_ops = np.ascontiguousarray(uccsd_pool(p.n_orb, p.n_alpha, p.n_beta), dtype=np.int32)
        for exc in (0, 1):
            q = vp()
            ok(lib.fsv_pool_create(ctypes.byref(q), plan, pool_ops.ctypes.data_as(I32), len(pool_ops), exc), "pool")
            th = np.ascontiguousarray(p.theta)
            e = ctypes.c_double()
            g = np.zeros(len(pool_ops))
            for _ in range(2):
                ok(lib.fsv_pool_gradients(q, dp(th), psi.p, lam.p, ctypes.byref(e), dp(g)), "pool grads")
            ok(lib.fsv_pool_destroy(q), "pool destroy")
        psi.free()
        lam.free()
        ok(lib.fsv_plan_destroy(plan), "destroy")
    # a pool destroyed after its plan (the order a garbage collector may take)
    p = config("C1")
    plan = make_plan(p)
    q = vp()
    ops = np.ascontiguousarray(p.ops)
    ok(lib.fsv_pool_create(ctypes.byref(q), plan, ops.ctypes.data_as(I32), len(ops), 0), "pool")
    ok(lib.fsv_plan_destroy(plan), "destroy")
    th = np.ascontiguousarray(p.theta)
    e = ctypes.c_double()
    g = np.zeros(len(ops))
    buf = Dev(1 << 12)
    buf2 = Dev(1 << 12)
    if lib.fsv_pool_gradients(q, dp(th), buf.p, buf2.p, ctypes.byref(e), dp(g)) != -4:
        raise RuntimeError("a pool whose plan is destroyed must refuse to run")
    buf.free()
    buf2.free()
    ok(lib.fsv_pool_destroy(q), "pool destroy after plan")
    # multi-determinant starts
    for ordering in (0, 1):
        p = config("C2", ordering)
        for engine in (0, 1):
            plan = make_plan(p, engine=engine)
            idx = np.array([0], dtype=np.uint64)
            keep = []
            cp = cproblem(p, 0, keep)
            del cp
            ok(lib.fsv_set_initial_state(plan, 0, None, None), "init")
            ok(lib.fsv_plan_destroy(plan), "destroy")
            del idx


def suite_batch():
    shapes = [(4, 2, 3), (6, 3, 10), (8, 4, 26), (8, 1, 5), (10, 7, 20), (12, 6, 40), (12, 4, 30),
              (10, 5, 0), (14, 7, 25), (6, 6, 0), (16, 9, 30)]
    probs = []
    for i, (n, ne, k) in enumerate(shapes):
        p = random_problem(n, ne, k if k else None, seed=700 + i, theta_std=0.3, replace=True, ordering=i % 2)
        if k == 0:
            p.ops = np.zeros((0, 4), dtype=np.int32)
            p.theta = np.zeros(0)
        probs.append(p)
    for mode in ("phased", "persistent", "packets"):
        for sigma in ("lds", "direct", "global"):
            for same_spin in ("dense", "sparse"):
                env = {"FSV_BATCH_MODE": mode}
                if sigma != "lds":
                    env["FSV_BATCH_SIGMA"] = sigma
                if same_spin == "sparse":
                    env["FSV_BATCH_SAME_SPIN"] = "sparse"
                print("batch", env, flush=True)
                with_env(env, lambda: run_batch(probs))
    with_env({"FSV_BATCH_MODE": "packets"}, lambda: run_batch(batch_config(), tune=True))


def run_batch(probs, tune=False):
    keep = []
    arr = (CProblem * len(probs))()
    for i, p in enumerate(probs):
        arr[i] = cproblem(p, 0, keep)
    b = vp()
    live0 = stub.hip_stub_live_device_bytes()
    ok(lib.fsv_batch_create(ctypes.byref(b), arr, len(probs), None), "batch create")
    if stub.hip_stub_live_device_bytes() - live0 != lib.fsv_batch_bytes(b):
        raise RuntimeError("fsv_batch_bytes does not match the batch's allocations")
    arena = Dev(lib.fsv_batch_arena_bytes(b))
    arena2 = Dev(lib.fsv_batch_arena_bytes(b))
    th = np.ascontiguousarray(np.concatenate([p.theta for p in probs]) if probs else np.zeros(0))
    e = np.zeros(len(probs))
    g = np.zeros(max(th.size, 1))
    for a in (arena, arena, arena2):
        ok(lib.fsv_batch_energy_grad(b, dp(th), a.p, dp(e), dp(g)), "batch eval")
    if tune:
        rep = ctypes.c_char_p()
        ok(lib.fsv_batch_autotune(b, arena.p, ctypes.byref(rep)), "batch autotune")
        ok(lib.fsv_batch_energy_grad(b, dp(th), arena.p, dp(e), dp(g)), "batch eval")
    ok(lib.fsv_batch_destroy(b), "batch destroy")
    arena.free()
    arena2.free()
    if stub.hip_stub_live_device_bytes() != live0:
        raise RuntimeError("the batch left device memory behind")


def suite_c3():
    p = config("C3")
    for engine in (0, 1):
        print("C3", engine, flush=True)
        exercise_plan(p, engine=engine, stages=False)


def suite_placement():
    # 20 qubits: packet runs of a few hundred packets, placed by XCD; every
    # XCD's range is padded to the same length, so a run's packet count is a
    # multiple of 8, and the whole plan still passes its own program checks
    p = random_problem(20, 10, 80, seed=1211, theta_std=0.4, replace=True, ordering=1)
    plan = make_plan(p)
    k = p.n_ops
    start = np.zeros(k, np.int32)
    tiles = np.zeros(k, np.int32)
    ok(lib.fsv_plan_runs(plan, 1, start.ctypes.data_as(I32), tiles.ctypes.data_as(I32)), "runs")
    placed = [int(t) for t in tiles if t >= 64]
    if not placed or any(t % 8 for t in placed):
        raise RuntimeError(f"packet counts of placed runs: {sorted(set(placed))}")
    print("placement", len(set(int(start[t]) for t in range(k) if tiles[t] > 0)), "packet runs", flush=True)
    ok(lib.fsv_plan_destroy(plan), "plan_destroy")
    exercise_plan(p, stages=False, extras=False)


SUITES = {"sigma": suite_sigma, "parity": suite_parity, "pools": suite_pools, "batch": suite_batch,
          "c3": suite_c3, "placement": suite_placement}

if __name__ == "__main__":
    for name in sys.argv[1:]:
        SUITES[name]()
        gc.collect()
    live = stub.hip_stub_live_device_bytes()
    handles = stub.hip_stub_live_handles()
    print(f"replay done: {stub.hip_stub_launches()} launches, {stub.hip_stub_replays()} graph replays, "
          f"{live} device bytes and {handles} handles still live", flush=True)
    if live or handles:
        raise SystemExit("device memory or handles leaked")
