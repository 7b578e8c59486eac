#!/usr/bin/env python3
"""Benchmark of the D-VQLS hot path on one MI355X.

Workload: n = 10 tridiagonal Toeplitz system A = tridiag(-0.45, 1, -0.45)
(N = 1024), b = |+>^10, FWHT Pauli decomposition pruned at tau = 0.01
(L = 64 strings), ansatz of 4 layers RY + CZ ladder (40 angles), local cost:
2(n+1)L^2 = 90,112 Hadamard-test circuits per cost evaluation.

One timed step = one VQLS iteration of the fast form:
  every circuit of the cost evaluation simulated with complex64 state
  vectors (float64 accumulation of the terms into the cost), the adjoint
  gradient (complex64 states) and the gradient-descent update.
The plain form (complex128 states, gradient by the parameter-shift rule:
(2P + 1) x 90,112 circuits per iteration) is timed beside it.

Prints one JSON line.  `value` is circuits of the cost evaluation completed
per second of whole-iteration wall time of the fast form.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "circuits/s + s/VQLS-iter @ n=10 L=64: FP32+adjoint+warm-start vs plain FP64"
FP32_ALU_PEAK = 78.6   # TFLOP/s: 256 CU x 4 SIMD x 16 lanes x FMA (2 flop) x 2.4 GHz, non-packed
FP64_ALU_PEAK = 78.6   # TFLOP/s: MI355X float64 vector peak
N_QUBITS, LAYERS, TAU, DIAG, OFFDIAG, ETA = 10, 4, 0.01, 1.0, -0.45, 0.05


def circuit_flops(n: int, layers: int) -> int:
    """Algorithmic float operations of one literal circuit on 2^(n+1)
    amplitudes: 6 per amplitude per RY (real 2x2 rotation of a complex
    amplitude), 4 per amplitude for the final ancilla H, 4 per amplitude for
    the <Z> accumulation; Pauli strings, CZ and X are sign/permutation only."""
    return (1 << (n + 1)) * (6 * n * layers + 4 + 4)


def cpu_baseline(seconds: float):
    """The oracle's gate-by-gate circuits on the host (one core), on a bounded
    sample of the same evaluation (real and imaginary circuits of beta and
    delta terms in the order of the evaluation, strided)."""
    import numpy as np

    from oracle import circuit as qc
    from oracle import pauli as op
    from workloads import theta_uniform, toeplitz

    n, layers = N_QUBITS, LAYERS
    C = op.decompose_fwht(toeplitz(n, DIAG, OFFDIAG))
    keep = op.select_tau(C, TAU)
    _, xs, zs = op.kept_terms(C, keep)
    L = len(keep)
    th = theta_uniform(n * layers, seed=0)
    total = 2 * (n + 1) * L * L
    done = 0
    t0 = time.perf_counter()
    c = 0
    while time.perf_counter() - t0 < seconds:
        part, u = c & 1, (c >> 1)
        jj, lm = divmod(u, L * L)
        l, m = divmod(lm, L)
        sl, sm = (int(xs[l]), int(zs[l])), (int(xs[m]), int(zs[m]))
        if jj == 0:
            qc.beta_circuit(th, n, layers, "cz", sl, sm, bool(part))
        else:
            qc.delta_circuit(th, n, layers, "cz", sl, sm, jj - 1, bool(part))
        done += 1
        c = (c + 7919) % total
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "circuits/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} of the {total} circuits of one n=10 L=64 cost evaluation, "
                      f"gate by gate in NumPy float64, {el:.1f} s on one core"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (calibrates HBM counters)")
    ap.add_argument("--no-fwht", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2604_14435_amd import api
    from workloads import theta_uniform, toeplitz

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n, layers = N_QUBITS, LAYERS
    an = api.AnsatzSpec(n, layers, "cz")
    P = an.P
    A = torch.from_numpy(toeplitz(n, DIAG, OFFDIAG)).to(dev)

    # one-off preprocessing: decomposition + pruning (Algorithm 1 Steps 1-2)
    coeffs, strings, ferr = api.pauli_decompose(A, tau=TAU)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(5):
        coeffs, strings, ferr = api.pauli_decompose(A, tau=TAU)
    torch.cuda.synchronize()
    decompose_ms = (time.perf_counter() - t) / 5 * 1e3
    L = coeffs.shape[0]
    circuits = api.circuit_count(n, L, "local")

    theta0 = torch.from_numpy(theta_uniform(P, seed=0)).to(dev)
    beta = torch.empty((1, L, L), dtype=torch.complex128, device=dev)
    delta = torch.empty((1, n, L, L), dtype=torch.complex128, device=dev)
    C = torch.empty(1, dtype=torch.float64, device=dev)
    parts = torch.empty((1, 2), dtype=torch.complex128, device=dev)
    Ca = torch.empty(1, dtype=torch.float64, device=dev)
    grad = torch.empty((1, P), dtype=torch.float64, device=dev)

    ev = []

    def fast_step(theta, record):
        if record:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
        api.vqls_terms(an, theta, strings, "local", "f32", out=(beta, delta))
        if record:
            e1.record()
            ev.append((e0, e1))
        api.vqls_cost(coeffs, n, "local", beta, delta, out=(C, parts))
        api.vqls_grad_adjoint(an, theta, coeffs, strings, "local", "f32", out=(Ca, grad))
        api.gd_step(theta, grad, ETA)

    theta = theta0.clone()
    for _ in range(args.warmup):
        fast_step(theta, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fast_step(theta, True)
    torch.cuda.synchronize()
    fast_s = (time.perf_counter() - t0) / args.steps
    kern_ms = sum(a.elapsed_time(b) for a, b in ev) / len(ev)

    # plain form: complex128 circuits + parameter-shift gradient
    ws = api.ShiftWorkspace(an, L, "local", dev)
    Cp = torch.empty(1, dtype=torch.float64, device=dev)
    gp = torch.empty(P, dtype=torch.float64, device=dev)
    thp = theta0.clone()

    def plain_step(th):
        api.vqls_grad_shift(an, th, coeffs, strings, "local", "f64", workspace=ws, out=(Cp, gp))
        api.gd_step(th, gp, ETA)

    plain_step(thp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.plain_steps):
        plain_step(thp)
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / args.plain_steps
    plain_circuits = (2 * P + 1) * circuits

    # the prefix-shared execution of the same evaluation (reported separately)
    api.vqls_terms(an, theta0, strings, "local", "f32", exec_="shared", out=(beta, delta))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        api.vqls_terms(an, theta0, strings, "local", "f32", exec_="shared", out=(beta, delta))
    e1.record()
    torch.cuda.synchronize()
    shared_ms = e0.elapsed_time(e1) / args.steps

    # FWHT decomposition of the dense random symmetric 4096 x 4096 matrix
    fwht = None
    if not args.no_fwht:
        from workloads import random_symmetric
        A12 = torch.from_numpy(random_symmetric(12, seed=0)).to(dev)
        c12 = api.pauli_decompose_dense(A12)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record()
        for _ in range(reps):
            api.pauli_decompose_dense(A12)
        e1.record()
        torch.cuda.synchronize()
        fwht_ms = e0.elapsed_time(e1) / reps
        alg_bytes = (8 + 16) * 4 ** 12
        fwht = {"bound": "hbm", "achieved": round(alg_bytes / (fwht_ms * 1e-3) / 1e9, 1), "peak": 8000.0,
                "unit": "GB/s", "frac": round(alg_bytes / (fwht_ms * 1e-3) / 8e12, 4), "traffic": None,
                "kernel": "k_fwht_pass1 + k_fwht_pass2 (n=12 dense)", "avg_ms": round(fwht_ms, 4),
                "algorithmic_bytes": alg_bytes}
        del A12, c12

    # float32 form vs the float64 path at theta0 (terms, cost, gradient)
    b32, d32 = api.vqls_terms(an, theta0, strings, "local", "f32")
    b64, d64 = api.vqls_terms(an, theta0, strings, "local", "f64")
    c32, _ = api.vqls_cost(coeffs, n, "local", b32, d32)
    c64, _ = api.vqls_cost(coeffs, n, "local", b64, d64)
    _, g32 = api.vqls_grad_adjoint(an, theta0, coeffs, strings, "local", "f32")
    _, g64 = api.vqls_grad_adjoint(an, theta0, coeffs, strings, "local", "f64")
    errors = {
        "beta_max_abs": float(torch.max(torch.abs(b32 - b64)).item()),
        "delta_max_abs": float(torch.max(torch.abs(d32 - d64)).item()),
        "cost_abs": float(abs(c32.item() - c64.item())),
        "grad_max_abs": float(torch.max(torch.abs(g32 - g64)).item()),
        "reference": "complex128 GPU path (itself within 1e-12 of the CPU oracle)",
    }

    flops = circuit_flops(n, layers) * circuits
    achieved = flops / (kern_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_ALU_PEAK,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_ALU_PEAK, 4), "traffic": None,
                "kernel": "k_terms_fast<float,10>", "avg_kernel_ms": round(kern_ms, 4),
                "flops_per_launch": flops}

    out = {
        "metric": METRIC,
        "value": round(circuits / fast_s, 1),
        "unit": "circuits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fast_s * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "toeplitz_n10_L64", "n": n, "L": int(L), "layers": layers,
                   "entangler": "cz", "cost": "local", "b": "plus", "tau": TAU,
                   "circuits_per_evaluation": int(circuits), "parallelism": "1 GPU"},
        "s_per_vqls_iter": {"fp32_adjoint": round(fast_s, 6), "plain_fp64_shift": round(plain_s, 6)},
        "circuits_per_s": {"fp32_adjoint": round(circuits / fast_s, 1),
                           "plain_fp64_shift": round(plain_circuits / plain_s, 1)},
        "per_iter_speedup": round(plain_s / fast_s, 2),
        "decompose_ms": round(decompose_ms, 4),
        "frobenius_error": round(ferr, 6),
        "error_fp32_vs_fp64": errors,
        "roofline": roofline,
        "prefix_shared": {"terms_ms": round(shared_ms, 4),
                          "circuits_per_s": round(circuits / (shared_ms * 1e-3), 1),
                          "note": "same circuits and results; the ansatz prefix simulated once per wavefront"},
        "roofline_fwht": fwht,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
