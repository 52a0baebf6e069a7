"""Benchmark of the hot path: one [H, O] + merge + truncate on one MI355X.

Workload (the commutator microbenchmark): open N=64 chain,
H = sum Z_i Z_{i+1} + 1.05 sum X_i + 0.5 sum Z_i (191 strings), O = 2^20
distinct random strings with support on <= 10 contiguous sites and complex
N(0,1) coefficients (seed 20241009), truncation to length <= 12 and the top
2^20 strings by |c|.  A step is one full pauli_commutator call with its
inputs resident in HBM.  Throughput is counted in (H string, O string) pairs
per second, the loop count of the paper's Alg. 1.

Prints one JSON line.  Single GPU only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Pauli string products/sec in [H,O]+merge+truncate; b_n rel err vs FP64"
HBM_PEAK_GBS = 8000.0
R_BYTES = 32  # one record at N=64 in FP64: 16 B key + 16 B complex coefficient


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 20 calls; 40 Lanczos / 200 RK4 steps for "
                         "the other workloads)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--count", type=int, default=1 << 20, help="strings in O")
    ap.add_argument("--cpu-sample", type=int, default=1 << 17,
                    help="O strings given to the single-threaded CPU oracle timing (0: skip "
                         "every CPU baseline)")
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="host threads of the full-size CPU oracle run (at most the usable CPUs)")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--workload", default="commutator",
                    choices=["commutator", "lanczos-split", "rk4-tfim", "lanczos-small", "moments",
                             "noisy-xxz", "lanczos-ts", "surrogate"],
                    help="commutator: the benchmark line (default); the others run the "
                         "Lanczos precision-split, RK4, small-Lanczos, spectral-moment, "
                         "noisy-diffusion, translation-symmetric Lanczos and b_n-surrogate "
                         "configurations and print their own result line")
    ap.add_argument("--max-strings", type=int, default=0,
                    help="truncation M for lanczos-split / rk4-tfim (0: the configuration's)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain elementwise copy of BYTES bytes 5 times "
                         "(reference for the HBM traffic counters) and exit")
    return ap.parse_args()


def kernel_source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hpp", "select.hpp", "device_common.hpp", "engine.hip"):
        with open(os.path.join(ROOT, "paper_2410_09654_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "commutator_microbench_traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("source_sha") != kernel_source_sha() or kernel not in t["kernels"]:
        return None
    k = t["kernels"][kernel]
    cal = t["copy_calibration"]
    return {"fetch_bytes": round(k["fetch_bytes"]), "write_bytes": round(k["write_bytes"]),
            "total_bytes": round(k["fetch_bytes"] + k["write_bytes"]),
            "fetch_factor": round(cal["fetch_factor"], 4), "write_factor": round(cal["write_factor"], 4),
            "read_bytes_by_request_size": round(k["read_bytes_by_request_size"]),
            "write_bytes_by_request_size": round(k["write_bytes_by_request_size"])}


def host_info(threads_used: int | None = None) -> dict:
    """nproc, CPU model and GPU name of the machine running the benchmark."""
    import torch
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    info = {"nproc": os.cpu_count(), "cpus_usable": len(os.sched_getaffinity(0)),
            "cpu_model": model,
            "gpu": torch.cuda.get_device_name(0) if torch.cuda.is_available() else None}
    if threads_used is not None:
        info["threads_used"] = threads_used
    return info


def measured_copy_gbs(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """HBM bandwidth of a plain device-to-device copy of `nbytes` (read + write
    counted), timed with events: the practical ceiling beside the 8 TB/s spec."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def cpu_threads(args) -> int:
    return max(1, min(args.cpu_threads, len(os.sched_getaffinity(0))))


def calibrate_copy(nbytes: int):
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.mul(src, 1.0, out=dst)  # elementwise kernel: reads and writes nbytes
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 5}), flush=True)


def step_roofline(tot: dict, wall: float, steps: int) -> dict:
    """Whole-step HBM roofline fraction: the algorithmic bytes of every engine
    pass of the timed steps (inputs + 2 records + 2 merged + output, at the
    record size; pauli_read_totals) over the wall time, against 8 TB/s."""
    gbs = tot["alg_bytes"] / wall / 1e9
    return {"bound": "hbm", "alg_bytes_per_step": tot["alg_bytes"] / max(steps, 1),
            "records_per_step": tot["emitted"] / max(steps, 1),
            "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def run_lanczos_split(args):
    """N=128 chain sum(XX+YY+0.5ZZ) + 0.3 sum r_i Z_i, O0 = sum X_i/sqrt(N),
    M = 2^23, 40 steps: FP64 and the FP32 + Kahan precision split side by side."""
    import torch
    import workloads as wl
    import paper_2410_09654_amd as pk
    steps = args.steps
    M = args.max_strings or (1 << 23)
    H_host, O0_host = wl.config_lanczos_split()
    H = pk.PauliOp.from_raw(128, H_host.x, H_host.z, H_host.coef)
    # the same H in reverse order: FP64 with another summation order, which
    # measures how far the truncated recursion itself amplifies rounding noise
    Hr = pk.PauliOp.from_raw(128, H_host.x[::-1], H_host.z[::-1], H_host.coef[::-1])
    # control: FP64 with H's coefficients perturbed by 2^-24 relative (FP32's
    # unit roundoff), to separate the recursion's sensitivity to the strings
    # kept at the cut from the precision split itself
    rs = np.random.default_rng(11).choice([-1.0, 1.0], size=len(H_host.coef))
    Hp = pk.PauliOp.from_raw(128, H_host.x, H_host.z, H_host.coef * (1.0 + rs * 2.0 ** -24))
    ws = pk.Workspace(1 << 30)
    res = {}
    for name, dt, Hn in (("f64", pk.PAULI_C128, H), ("f32_kahan", pk.PAULI_C64K, H),
                         ("f64_reversed_H", pk.PAULI_C128, Hr),
                         ("f64_perturbed_H", pk.PAULI_C128, Hp)):
        H = Hn
        O0 = pk.PauliOp.from_host(O0_host, dtype=dt, ws=ws)
        trunc = pk.Trunc(max_strings=M)
        prev, cur, b_prev = None, O0, 0.0
        bs, sizes, pairs, emitted = [], [], 0, 0
        torch.cuda.synchronize()
        pk.read_totals(reset=True)
        t0 = time.perf_counter()
        for _ in range(steps):
            pairs += H.size * cur.size
            nxt, b, broke = pk.lanczos_step(H, prev, cur, b_prev, trunc, ws=ws)
            emitted += pk.last_stats()["emitted"]
            bs.append(b)
            sizes.append(nxt.size)
            if broke:
                break
            prev, cur, b_prev = cur, nxt, b
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tot = pk.read_totals()
        res[name] = {"b": bs, "strings": sizes, "seconds": wall, "ms_per_step": 1e3 * wall / len(bs),
                     "pairs_per_s": pairs / wall, "emitted_per_s": emitted / wall,
                     "roofline_step": step_roofline(tot, wall, len(bs))}
    b64, b32, b64r = res["f64"]["b"], res["f32_kahan"]["b"], res["f64_reversed_H"]["b"]
    b64p = res["f64_perturbed_H"]["b"]
    m = min(len(b64), len(b32), len(b64r), len(b64p))
    rel = [abs(b32[k] - b64[k]) / abs(b64[k]) for k in range(m)]
    rel_r = [abs(b64r[k] - b64[k]) / abs(b64[k]) for k in range(m)]
    rel_p = [abs(b64p[k] - b64[k]) / abs(b64[k]) for k in range(m)]
    full = [k for k in range(m) if res["f64"]["strings"][k] < M]  # steps before the cut binds
    one_step = None
    if args.cpu_sample > 0:
        # one Lanczos step, oracle and GPU, FP64 and FP32 + Kahan, from the
        # oracle's own vectors after five steps at M = 2^12 (budget binding)
        import oracle
        one_step = {}
        for name, prec, dt in (("f64", oracle.F64, pk.PAULI_C128),
                               ("f32_kahan", oracle.F32K, pk.PAULI_C64K)):
            th = oracle.Trunc(max_strings=1 << 12)
            o0 = O0_host if prec == oracle.F64 else wl.HostOp(
                128, O0_host.x, O0_host.z, O0_host.coef.astype(np.complex64).astype(complex))
            prev, cur, b_prev = None, o0, 0.0
            for _ in range(5):
                nxt, b_prev_new, _ = oracle.lanczos_step(H_host, prev, cur, b_prev, th, prec)
                prev, cur, b_prev = cur, nxt, b_prev_new
            tc = time.perf_counter()
            oracle.lanczos_step(H_host, prev, cur, b_prev, th, prec)
            tcpu = time.perf_counter() - tc
            Hd = pk.PauliOp.from_raw(128, H_host.x, H_host.z, H_host.coef)
            pd = pk.PauliOp.from_host(prev, dtype=dt, ws=ws)
            cd = pk.PauliOp.from_host(cur, dtype=dt, ws=ws)
            pk.lanczos_step(Hd, pd, cd, b_prev, pk.Trunc(max_strings=1 << 12), ws=ws)
            torch.cuda.synchronize()
            tg = time.perf_counter()
            pk.lanczos_step(Hd, pd, cd, b_prev, pk.Trunc(max_strings=1 << 12), ws=ws)
            torch.cuda.synchronize()
            one_step[name] = {"strings": cur.n, "oracle_seconds": tcpu,
                              "gpu_seconds": time.perf_counter() - tg, "cores": 1}
    print(json.dumps({"workload": "lanczos precision split: N=128 XXZ(0.5) + 0.3 r_i Z_i, "
                                  "O0 = sum X_i/sqrt(N)", "steps": steps, "max_strings": M,
                      "b_rel_err_vs_f64": rel, "max_b_rel_err": max(rel) if rel else None,
                      "max_b_rel_err_untruncated_steps": max([rel[k] for k in full], default=None),
                      "f64_order_sensitivity": rel_r,
                      "max_f64_order_sensitivity": max(rel_r) if rel_r else None,
                      "f64_h_perturbation_2m24_sensitivity": rel_p,
                      "max_f64_h_perturbation_sensitivity": max(rel_p) if rel_p else None,
                      "max_h_perturbation_sensitivity_untruncated_steps":
                          max([rel_p[k] for k in full], default=None),
                      "one_step_M4096_from_oracle_state": one_step, "host": host_info(),
                      **res}), flush=True)


def run_rk4_tfim(args):
    """8x8 open TFIM (J=1, hx=2), O0 = Z at site (4,4), dt = 0.02, 200 steps,
    M = 2^22, length <= 16, keep = {O0}; S(t) = <O0, O(t)>."""
    import torch
    import workloads as wl
    import paper_2410_09654_amd as pk
    steps = args.steps
    M = args.max_strings or (1 << 22)
    H_host, O0_host = wl.config_rk4_tfim()
    H = pk.PauliOp.from_raw(64, H_host.x, H_host.z, H_host.coef)
    ws = pk.Workspace(1 << 30)
    O0 = pk.PauliOp.from_host(O0_host, ws=ws)
    trunc = pk.Trunc(max_len=16, max_strings=M, keep=O0)
    S, sizes, pairs = [1.0], [O0.size], 0
    cur = O0
    torch.cuda.synchronize()
    pk.read_totals(reset=True)
    t0 = time.perf_counter()
    for k in range(steps):
        pairs += 4 * H.size * cur.size  # lower bound: the stages grow beyond |O|
        cur = pk.rk4_step(H, cur, 0.02, trunc, ws=ws)
        S.append(pk.correlator(O0, cur, ws=ws).real)
        sizes.append(cur.size)
        if k % 50 == 49:
            print(f"rk4 step {k + 1}: {1e3 * (time.perf_counter() - t0) / (k + 1):.1f} ms/step",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tot = pk.read_totals()
    line = {"workload": "rk4 8x8 TFIM J=1 hx=2, O0 = Z(4,4), dt = 0.02",
            "steps": steps, "max_strings": M, "max_len": 16,
            "seconds": wall, "ms_per_step": 1e3 * wall / steps, "S": S,
            "strings": sizes, "roofline_step": step_roofline(tot, wall, steps),
            "host": host_info()}
    if args.cpu_sample > 0:
        # one RK4 step, oracle and GPU, from the oracle's own state after five
        # steps at M = 2^12 (budget binding; a full-M step takes minutes on the host)
        import oracle
        Ms = 1 << 12
        th = oracle.Trunc(max_len=16, max_strings=Ms, keep=O0_host)
        st = O0_host
        for _ in range(5):
            st = oracle.rk4_step(H_host, st, 0.02, th)
        tc = time.perf_counter()
        oracle.rk4_step(H_host, st, 0.02, th)
        tcpu = time.perf_counter() - tc
        sd = pk.PauliOp.from_host(st, ws=ws)
        tg_trunc = pk.Trunc(max_len=16, max_strings=Ms, keep=O0)
        pk.rk4_step(H, sd, 0.02, tg_trunc, ws=ws)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        pk.rk4_step(H, sd, 0.02, tg_trunc, ws=ws)
        torch.cuda.synchronize()
        line["one_step_M4096_from_oracle_state"] = {
            "strings": st.n, "oracle_seconds": tcpu, "gpu_seconds": time.perf_counter() - tg,
            "cores": 1}
    print(json.dumps(line), flush=True)


def run_lanczos_small(args):
    """N=12 chain, O0 = Z_1, 12 untruncated FP64 Lanczos steps, timed (the
    small operators make each step one library call at its host floor), with
    the oracle's recursion on the same steps beside it."""
    import torch
    import workloads as wl
    import paper_2410_09654_amd as pk
    H_host, O0_host, steps = wl.config_lanczos_small()
    H = pk.PauliOp.from_raw(12, H_host.x, H_host.z, H_host.coef)
    O0 = pk.PauliOp.from_host(O0_host)
    pk.lanczos(H, O0, steps)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bs, basis = pk.lanczos(H, O0, steps, keep_basis=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    counts = [B.size for B in basis[1:]]
    small = [int(np.sum(np.abs(B.to_host().coef) > 1e-12)) for B in basis[1:]]
    line = {"workload": "lanczos N=12 chain, O0 = Z_1", "b": bs, "strings": counts,
            "strings_above_1e-12": small, "seconds": wall, "ms_per_step": 1e3 * wall / len(bs)}
    if args.cpu_sample > 0:
        import oracle
        tc = time.perf_counter()
        bo = oracle.lanczos(H_host, O0_host, steps)
        line["oracle"] = {"seconds": time.perf_counter() - tc, "cores": 1,
                          "max_rel_diff_b": max(abs(a - b) / abs(b) for a, b in zip(bs, bo))}
    print(json.dumps(line), flush=True)


def run_moments(args):
    """Spectral moments mu_k = Tr(H^k)/2^N, k = 1..4, of the N=64 chaotic Ising
    chain (|H| = 191) by untruncated string products H^k = H H^(k-1) and the
    identity coefficient; the last product pairs 191 x |H^3| = 2.0e8 strings.
    The oracle computes mu_1..mu_3 beside it (mu_4 needs 2e8 records)."""
    import torch
    import workloads as wl
    import paper_2410_09654_amd as pk
    H_host = wl.ising_chain(64, hx=1.05, hz=0.5)
    H = pk.PauliOp.from_raw(64, H_host.x, H_host.z, H_host.coef)
    ws = pk.Workspace(1 << 30)
    kmax = 4
    for _ in range(max(args.warmup, 1)):
        pk.moments(H, kmax, ws=ws)
    steps = args.steps or 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        mus = pk.moments(H, kmax, ws=ws)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    # the last product alone
    P = H
    for _ in range(kmax - 2):
        P = pk.multiply(H, P, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        pk.multiply(H, P, ws=ws)
    torch.cuda.synchronize()
    t_last = (time.perf_counter() - t1) / steps
    st = pk.last_stats()
    pairs = H.size * P.size
    line = {"workload": "spectral moments Tr(H^k)/2^N, N=64 chaotic Ising chain (hx=1.05, hz=0.5), "
                        "k=1..4, untruncated products",
            "mu": [[m.real, m.imag] for m in mus], "ms_per_moments_call": wall * 1e3,
            "last_product": {"pairs": pairs, "ms": t_last * 1e3, "pairs_per_s": pairs / t_last,
                             "emitted": st["emitted"], "unique": st["unique"],
                             "passes": st["passes"]}}
    if args.cpu_sample > 0:
        import oracle
        tc = time.perf_counter()
        want = oracle.moments(H_host, 3)
        t_o = time.perf_counter() - tc
        # mu_4 = Tr(H^2 H^2)/2^N = ||H^2||^2 for Hermitian H
        mu4 = oracle.norm2(oracle.product(H_host, H_host))
        line["oracle"] = {"mu_1_3": [[m.real, m.imag] for m in want],
                          "seconds_mu_1_3": t_o, "cores": 1,
                          "max_abs_diff_mu_1_3": max(abs(a - b) for a, b in zip(mus[:3], want)),
                          "mu_4_as_norm2_of_H2": mu4,
                          "rel_diff_mu_4": abs(mus[3] - mu4) / abs(mu4)}
    print(json.dumps(line), flush=True)


def run_noisy_xxz(args):
    """Noisy diffusion on the periodic next-nearest-neighbour XXZ chain
    (N=30, delta=2, gamma=1/2): O0 = Z_1, dt=0.05, 200 RK4 steps (t = 10),
    M = 2^18 with O0 kept, depolarizing eps = 0.01; S(t), the two-point
    correlators S_{1-j}(t) and n(t) = sum_j S_{1-j}(t) (exp(-eps t) without
    truncation)."""
    import math
    import torch
    import workloads as wl
    import paper_2410_09654_amd as pk
    H_host, O0_host, probes_host = wl.config_noisy_xxz()
    n = H_host.n_qubits
    dt, steps, eps = 0.05, args.steps or 200, 0.01
    M = args.max_strings or (1 << 18)
    H = pk.PauliOp.from_raw(n, H_host.x, H_host.z, H_host.coef)
    O0 = pk.PauliOp.from_host(O0_host)
    probes = pk.PauliOp.from_raw(n, probes_host.x, probes_host.z, probes_host.coef)
    ws = pk.Workspace(1 << 30)
    pk.evolve_noisy(H, O0, dt, 2, M, eps, probes=probes, ws=ws)  # warm-up
    def progress(k, op):
        if k % 20 == 0:
            print(f"step {k}: {op.size} strings, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    O, S, P = pk.evolve_noisy(H, O0, dt, steps, M, eps, probes=probes, ws=ws, observe=progress)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nt = [float(np.sum(p).real) for p in P]
    line = {"workload": "noisy XXZnnn diffusion: N=30 periodic, delta=2, gamma=1/2, O0 = Z_1, "
                        "dt=0.05, eps=0.01, M=2^18 (O0 kept)",
            "steps": steps, "max_strings": M, "seconds": wall, "ms_per_step": 1e3 * wall / steps,
            "final_strings": O.size,
            "S": [float(v.real) for v in S[::10]],
            "S_1j_final": [float(v.real) for v in P[-1]],
            "n_t_over_exp": [nt[k] / math.exp(-eps * k * dt) for k in range(0, steps + 1, 20)],
            "max_abs_n_minus_exp": max(abs(nt[k] - math.exp(-eps * k * dt))
                                       for k in range(steps + 1))}
    if args.cpu_sample > 0:
        import oracle
        # one noisy step, oracle and GPU, from the oracle's own state after
        # four steps at M = 4096 (a full-M step would take minutes on one core)
        Ms = 4096
        hs, _, _ = oracle.evolve_noisy(H_host, O0_host, dt, 4, Ms, eps)
        print(f"oracle step from {hs.n} strings", file=sys.stderr, flush=True)
        tc = time.perf_counter()
        oracle.evolve_noisy(H_host, hs, dt, 1, Ms, eps)
        tcpu = time.perf_counter() - tc
        Os = pk.PauliOp.from_host(hs, ws=ws)
        pk.evolve_noisy(H, Os, dt, 1, Ms, eps, ws=ws)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        pk.evolve_noisy(H, Os, dt, 1, Ms, eps, ws=ws)
        torch.cuda.synchronize()
        tgpu = time.perf_counter() - tg
        line["step_from_oracle_state_M4096"] = {"strings": hs.n, "oracle_seconds": tcpu,
                                                "gpu_seconds": tgpu, "cores": 1}
    print(json.dumps(line), flush=True)


def run_lanczos_ts(args):
    """Lanczos recursion on translation-symmetric operators (Alg. 2) of the
    periodic chains of the paper's translation-symmetry figure, N = 50, each
    O0 given by its orbit representatives and normalised:
      XX:        H0 = {XX, YY},              O0 ~ sum_j X_j,                    50 steps;
      XXX:       H0 = {XX, YY, ZZ},          O0 ~ sum_j X_j Y_j+1 - Y_j X_j+1,  20 steps;
      chaotic:   H0 = {XX, -1.05 Z, 0.5 X},  O0 ~ sum_j 1.05 X_j X_j+1 + Z_j,   40 steps;
      chaotic with h_X = 0.1 in place of 0.5,                                   40 steps;
    at M = 2^20 (--max-strings), with the oracle beside it on 10 steps at
    M = 2^10."""
    import math
    import torch
    import workloads as wl
    import paper_2410_09654_amd as pk
    M = args.max_strings or (1 << 20)
    ws = pk.Workspace(1 << 30)
    n = 50
    XX = [(1.0, [("X", 1), ("X", 2)]), (1.0, [("Y", 1), ("Y", 2)])]
    runs = {
        "xx": (XX, [(1.0, [("X", 1)])], 50),
        "xxx": (XX + [(1.0, [("Z", 1), ("Z", 2)])],
                [(1.0, [("X", 1), ("Y", 2)]), (-1.0, [("Y", 1), ("X", 2)])], 20),
        "chaotic_hx0.5": ([(1.0, [("X", 1), ("X", 2)]), (-1.05, [("Z", 1)]), (0.5, [("X", 1)])],
                          [(1.05, [("X", 1), ("X", 2)]), (1.0, [("Z", 1)])], 40),
        "chaotic_hx0.1": ([(1.0, [("X", 1), ("X", 2)]), (-1.05, [("Z", 1)]), (0.1, [("X", 1)])],
                          [(1.05, [("X", 1), ("X", 2)]), (1.0, [("Z", 1)])], 40),
    }
    line = {"workload": "translation-symmetric Lanczos (Alg. 2 commutator), periodic N = 50",
            "max_strings": M}
    for name, (h_terms, o_terms, steps) in runs.items():
        H0h = wl.from_terms(n, h_terms)
        O0h = wl.from_terms(n, o_terms)
        O0h.coef /= math.sqrt(float(np.sum(np.abs(O0h.coef) ** 2)))  # no stabilizers: norm 1
        H0 = pk.PauliOp.from_raw(n, H0h.x, H0h.z, H0h.coef)
        O0 = pk.PauliOp.from_host(O0h, ws=ws)
        pk.lanczos_ts1d(H0, O0, 3, pk.Trunc(max_strings=M), ws=ws)  # warm-up
        sizes = [O0.size]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bs = pk.lanczos_ts1d(H0, O0, steps, pk.Trunc(max_strings=M), ws=ws,
                             observe=lambda k, O: sizes.append(O.size))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # pairs of one step: N |H0| translated H strings times the representatives of O_{n-1}
        pairs = n * H0.size * sum(sizes[:len(bs)])
        r = {"steps": len(bs), "b": bs, "strings": sizes[1:], "seconds": wall,
             "ms_per_step": 1e3 * wall / max(len(bs), 1), "pairs_per_s": pairs / wall}
        if args.cpu_sample > 0:
            import oracle
            tc = time.perf_counter()
            bo = oracle.lanczos_ts(H0h, O0h, 10, oracle.Trunc(max_strings=1 << 10))
            tcpu = time.perf_counter() - tc
            torch.cuda.synchronize()
            tg = time.perf_counter()
            bg = pk.lanczos_ts1d(H0, O0, 10, pk.Trunc(max_strings=1 << 10), ws=ws)
            torch.cuda.synchronize()
            r["oracle_10_steps_M1024"] = {
                "oracle_seconds": tcpu, "gpu_seconds": time.perf_counter() - tg, "cores": 1,
                "max_rel_diff_b": max(abs(a - b) / max(abs(b), 1e-300) for a, b in zip(bg, bo))}
        line[name] = r
        print(f"{name}: {len(bs)} steps in {wall:.2f} s", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


MLP_FWD_FLOP = 2 * (16 * 256 + 256 * 256 + 256 * 16)  # per window
MLP_TRAIN_FLOP = 3 * MLP_FWD_FLOP  # forward, input gradient, weight gradient


def run_surrogate(args):
    """b_n continuation network: 512 random couplings (hx ~ U[0.5,1.5],
    hz ~ U[0,1], seed 5) of the N=64 Ising chain with O0 = sum Z_i/sqrt(N),
    truncated Lanczos at M = 2^20; 64 held-out couplings (seed 55) computed
    to 30 steps and continued to 46 by the network, scored against their
    plain 46-step recursion.  Two trainings: on the 30-step runs as the
    configuration states (windows k = 1..14, targets beyond b_30 masked,
    continuation by two passes), and on 46-step runs."""
    import math
    import torch
    import workloads as wl
    import paper_2410_09654_amd as pk
    from paper_2410_09654_amd import surrogate as sg
    M = args.max_strings or (1 << 20)
    ws = pk.Workspace(1 << 30)

    def tables(couplings, steps):
        out = []
        for hx, hz in couplings:
            H = wl.ising_chain(64, hx=float(hx), hz=float(hz))
            O0 = wl.single_site_sum(64, "Z", 1 / math.sqrt(64))
            Hd = pk.PauliOp.from_raw(64, H.x, H.z, H.coef)
            out.append(pk.lanczos(Hd, pk.PauliOp.from_host(O0, ws=ws), steps,
                                  pk.Trunc(max_strings=M), ws=ws))
        torch.cuda.synchronize()
        return np.array(out)

    t0 = time.perf_counter()
    train = tables(zip(*wl.surrogate_couplings(512, seed=5)), 46)
    t_gen = time.perf_counter() - t0
    cpl = list(zip(*wl.surrogate_couplings(64, seed=55)))
    t0 = time.perf_counter()
    short = tables(cpl, 30)
    t1 = time.perf_counter()
    held = tables(cpl, 46)
    t_lanczos16 = (time.perf_counter() - t1) - (t1 - t0)
    truth = held[:, 30:46]
    err = lambda p: float(np.mean(np.abs(p - truth) / truth))
    epochs, batch = 100, 256

    def fit(n_train, n_slots):
        """Train on the first n_train coefficients of every training run
        (targets masked beyond them) and continue b_1..b_30 to b_46 with
        n_slots output slots per network pass."""
        x, t, mask = sg.make_windows(train[:, :n_train], n_train)
        net = sg.BnSurrogate(seed=0, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = net.train(x.cuda(), t.cuda(), mask.cuda(), epochs=epochs, batch=batch, lr=1e-3)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        t0 = time.perf_counter()
        pred = sg.predict_continuation(net, short, 30, 46, n_slots=n_slots)
        torch.cuda.synchronize()
        t_mlp = time.perf_counter() - t0
        flops = MLP_TRAIN_FLOP * x.shape[0] * epochs
        return {"train_windows": int(x.shape[0]), "supervised_targets": int(mask.sum()),
                "held_out_mean_rel_err_mlp": err(pred),
                "per_step_rel_err_mlp": [float(v) for v in np.mean(np.abs(pred - truth) / truth,
                                                                    axis=0)],
                "loss_curve": hist[::10] + [hist[-1]], "training_seconds": t_train,
                "mlp_continuation_seconds": t_mlp, "training_tflops": flops / t_train / 1e12,
                "training_frac_of_bf16_peak": flops / t_train / 2.5e15}

    # as configured: 30-step training runs, windows k = 1..14 with the targets
    # beyond b_30 masked, continuation in two passes (slots 1..14, then 1..2)
    configured = fit(30, 14)
    # variant: 46-step training runs, so every output slot sees supervision
    deep = fit(46, 16)
    print(json.dumps({
        "workload": "b_n surrogate: N=64 Ising chain, 512 train / 64 held-out couplings, "
                    "truncated Lanczos at M=2^20, 16 -> 256 -> 256 -> 16 GELU",
        "max_strings": M, "epochs": epochs, "batch": batch,
        "held_out_mean_rel_err": {"mlp_30_step_training": configured["held_out_mean_rel_err_mlp"],
                                  "mlp_46_step_training": deep["held_out_mean_rel_err_mlp"],
                                  "constant_b30": err(sg.baseline_constant(short, 30, 46)),
                                  "linear_fit_b15_b30": err(sg.baseline_linear(short, 30, 46))},
        "as_configured_30_step_runs": configured, "variant_46_step_runs": deep,
        "seconds": {"training_tables_46_steps": t_gen, "lanczos_steps_31_46": t_lanczos16},
        "host": host_info()}), flush=True)


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the engine has no multi-GPU path; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.steps is None:
        args.steps = {"commutator": 20, "lanczos-split": 40, "rk4-tfim": 200}.get(args.workload, 0)
    if args.workload != "commutator":
        import torch
        import numpy as np  # noqa: F401
        globals()["np"] = np
        torch.cuda.set_device(0)
        {"lanczos-split": run_lanczos_split, "rk4-tfim": run_rk4_tfim,
         "lanczos-small": run_lanczos_small, "surrogate": run_surrogate,
         "moments": run_moments, "noisy-xxz": run_noisy_xxz,
         "lanczos-ts": run_lanczos_ts}[args.workload](args)
        return
    import torch
    import workloads as wl
    import paper_2410_09654_amd as pk

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    H_host, O_host = wl.config_commutator_bench(args.count)
    max_len, max_strings = 12, args.count
    H = pk.PauliOp.from_raw(64, H_host.x, H_host.z, H_host.coef)
    # room for the records of one pass from the first call on (a smaller
    # workspace makes the first call grow it and lay the pass out again)
    ws = pk.Workspace(4 << 30)
    O = pk.PauliOp.from_host(O_host, ws=ws)
    trunc = pk.Trunc(max_len=max_len, max_strings=max_strings)
    out = pk.PauliOp(64, max_strings + 16)

    for _ in range(max(args.warmup, 1)):
        pk.commutator(H, O, trunc, out=out, ws=ws)
    stats = pk.last_stats()

    # algorithmic bytes per launch (records of R bytes)
    nO, pe, u, m_out = O.size, stats["emitted"], stats["survivors"], stats["output"]
    alg_bytes = {
        "k_emit_count": nO * R_BYTES,
        "k_emit_scatter": (nO + pe) * R_BYTES,
        "k_merge": (pe + u) * R_BYTES,
        "k_write_out": (u + m_out) * R_BYTES,
    }

    # Per-kernel breakdown: an untimed pass with HIP events around every
    # kernel (the events themselves add about 8 us per launch, so they stay
    # out of the timed region), which also names the dominant kernel.
    kernel_timing = not args.no_kernel_timing
    per_kernel, dom = {}, None
    if kernel_timing:
        pk.profile_enable(True)
        for _ in range(min(args.steps, 10)):
            pk.commutator(H, O, trunc, out=out, ws=ws)
        torch.cuda.synchronize()
        per_kernel = {k: {"launches": c, "avg_ms": ms / c, "total_ms": ms}
                      for k, (c, ms) in pk.profile_read().items()}
        dom = max((k for k in per_kernel if k in alg_bytes), key=lambda k: per_kernel[k]["total_ms"])
        # timed region: events around the dominant kernel only, on the stream
        # the library launches on (the current torch stream)
        pk.profile_enable(True, only=[dom])
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        pk.commutator(H, O, trunc, out=out, ws=ws)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    live = pk.profile_read() if kernel_timing else {}
    pk.profile_enable(False)
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    pairs = H.size * O.size
    value = pairs * args.steps / wall

    roofline = None
    if dom is not None and dom in live:
        c, ms = live[dom]
        avg_s = ms / c * 1e-3
        achieved = alg_bytes[dom] / avg_s / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(dom), "alg_bytes_per_launch": alg_bytes[dom],
                    "avg_ms_timed_region": ms / c, "launches_timed_region": c}
        # merge + truncate stage: every kernel after the scatter (the
        # emission stage is H preparation, the count pass, its two scans and
        # the scatter), from the per-kernel pass
        np_steps = min(args.steps, 10)
        emission = ("k_prep_h", "k_mix_keys", "k_fill_u32", "k_emit_count", "k_scan_cols",
                    "k_scan_bins", "k_emit_scatter")
        mt_ms = sum(per_kernel[k]["total_ms"] for k in per_kernel
                    if k not in emission) / np_steps
        mt_bytes = (pe + 2 * u + m_out) * R_BYTES
        roofline["merge_truncate"] = {"ms_per_step": round(mt_ms, 4),
                                      "alg_bytes": mt_bytes,
                                      "achieved": round(mt_bytes / (mt_ms * 1e-3) / 1e9, 1),
                                      "frac": round(mt_bytes / (mt_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    if roofline is not None:
        copy = measured_copy_gbs()
        roofline["measured_copy_GBs"] = round(copy, 1)
        roofline["frac_of_measured_copy"] = round(roofline["achieved"] / copy, 4)

    cpu = None
    if args.cpu_sample > 0:
        import oracle
        # the whole workload on the host cores: O in chunks over the threads
        # (the C oracle as it stands, one call per chunk), added by linearity,
        # then the oracle's truncation
        nt = cpu_threads(args)
        tc0 = time.perf_counter()
        C = oracle.commutator_chunked(H_host, O_host, threads=nt, chunks=4 * nt)
        oracle.truncate(C, oracle.Trunc(max_len=max_len, max_strings=max_strings))
        tc = time.perf_counter() - tc0
        del C
        # single thread on a sample (the paper's one-core setting)
        n = min(args.cpu_sample, O_host.n)
        sub = wl.HostOp(64, O_host.x[:n], O_host.z[:n], O_host.coef[:n])
        ts0 = time.perf_counter()
        C1 = oracle.commutator(H_host, sub)
        oracle.truncate(C1, oracle.Trunc(max_len=max_len, max_strings=n))
        ts = time.perf_counter() - ts0
        cpu = {"value": pairs / tc, "unit": "products/s", "cores": nt, "kind": "oracle",
               "sample": f"the whole workload: all {O_host.n} O strings ({pairs} pairs) in "
                         f"{4 * nt} chunks over {nt} threads, added by linearity, then "
                         f"truncate (length <= {max_len}, top {max_strings}); {tc:.1f} s",
               "single_thread": {"value": H_host.n * n / ts, "cores": 1,
                                 "sample": f"first {n} O strings ({H_host.n * n} pairs), "
                                           f"commutator + truncate, {ts:.1f} s"},
               "host": host_info(nt)}

    line = {
        "metric": METRIC, "value": value, "unit": "products/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "commutator microbenchmark: N=64 chain, |H|=191, |O|=2^20 random "
                               "strings of support <= 10, one [H,O] + merge + truncate "
                               "(length <= 12, top 2^20)",
                   "n_qubits": 64, "H_strings": H.size, "O_strings": O.size,
                   "max_len": max_len, "max_strings": max_strings, "seed": 20241009},
        "emitted": pe, "unique": stats["unique"], "output": m_out,
        "emitted_per_s": pe * args.steps / wall,
        "gpu_event_ms_per_step": ev0.elapsed_time(ev1) / args.steps,
        "kernels": per_kernel,
        "kernels_note": "per-kernel events in an untimed pass of min(steps, 10) steps; "
                        "the timed region times only the roofline kernel",
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
