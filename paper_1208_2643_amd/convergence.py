"""Convergence study of Sec. 4.1 (Tables 1 and 2) on the GPU path.

    python -m paper_1208_2643_amd.convergence [--scheme 1|2] [--max-n 512]

Domain (0, 32)^2, eps = 0.025, beta = 0.9, M = 1, t_f = 10, the initial data
of the convergence tests (eq. initial-data).  Refinement paths: s = 0.05 h
(second-order scheme, Table 2) and s = 0.025 h^2 (first-order scheme,
Table 1).  For Table 1 the step runs the damped-wave form of the authors'
earlier work (beta = M = 1/0.9 in the form stepped here): that form reproduces
the table's printed first row; beta = 0.9, M = 1 does not.  Each grid is
stepped to t_f by the library (FP64, extrapolated guess); the reported
difference between the solutions on grids h and h/2 is the root-mean-square
of (2x2 average of the h/2 solution) - (h solution), with the average taken
by the library's restriction operator.

Cycle and tolerance per grid.  On 256^2 and finer grids of these refinement
paths the red-black collective Gauss-Seidel smoother of App. B is unstable on
its own (the residual grows by orders of magnitude per sweep, the CPU oracle
alike) and V(2,2) cycles diverge; V(0,1) cycles (one red-black pass after the
coarse-grid correction) converge in 8-14 cycles per step there.  So grids up
to 128^2 run V(2,2) and finer ones V(0,1), unless the smoother is
under-relaxed (omega < 1, e.g. 0.8), which makes V(2,2) converge on every
grid of both paths (9-12 cycles per step); the residual tolerance is 1e-11,
and 3e-11 on 512^2, where the FP64 residual of the first-order scheme
(s = 0.025 h^2) levels off near 2e-11.  There the extrapolated guess often
meets that tolerance without a cycle (its residual is at the floor too), and
the 102 400 steps of unsolved guesses drift by 1e-4; the previous step's phi
as the guess always leaves a residual above the floor, so every step is
solved.  A grid whose solve fails is reported with its error instead of a
difference.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def cycle_for(N: int, scheme: int, omega: float = 1.0):
    """(nu1, nu2, tol, guess) of the solves on an N x N grid of these
    refinement paths (guess 1: extrapolated, 0: the previous step's phi).
    With an under-relaxed smoother (omega < 1) every grid runs V(2,2)."""
    tol, guess = (1e-11, 1) if N <= 256 else (3e-11, 0 if scheme == 1 else 1)
    if N <= 128 or omega != 1.0:
        return 2, 2, tol, guess
    return 0, 1, tol, guess


def final_state(N: int, scheme: int, tol: float = None, omega: float = 1.0):
    """phi at t_f = 10 on an N x N grid (a GPU tensor) and the run's statistics
    (omega: the smoother's relaxation factor)."""
    import torch
    from . import api, inputs
    h = 32.0 / N
    if scheme == 2:
        s = 0.05 * h
        beta, M = 0.9, 1.0
    else:
        s = 0.025 * h * h
        beta, M = 1.0 / 0.9, 1.0 / 0.9
    steps = int(round(10.0 / s))
    nu1, nu2, tol_n, guess = cycle_for(N, scheme, omega)
    tol = tol_n if tol is None else tol
    p = api.Params(eps=0.025, beta=beta, M=M, h=h, dt=s, scheme=scheme)
    st = api.Stepper(N, N, p, tol=tol, energy=0, max_cycles=300, nu1=nu1, nu2=nu2, guess=guess,
                     omega=omega)
    phi = torch.from_numpy(inputs.paper_initial_data(N, N)).cuda()
    prev = phi.clone()
    psi = torch.zeros_like(phi)
    nxt = torch.empty_like(phi)
    t0 = time.perf_counter()
    cycles = 0
    for k in range(steps):
        _, info = st.step(phi, prev, psi, nxt)
        cycles += info.n_cycles
        prev, phi, nxt = phi, nxt, prev
        if (k + 1) % 20000 == 0:
            print(f"[convergence] N = {N}: {k + 1}/{steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    st.close()
    return phi, {"N": N, "h": h, "s": s, "steps": steps, "cycle": f"V({nu1},{nu2})", "tol": tol,
                 "guess": "extrapolated" if guess == 1 else "previous", "omega": omega,
                 "vcycles_per_step": cycles / steps, "seconds": time.perf_counter() - t0}


def table(scheme: int, sizes=(32, 64, 128, 256, 512), omega: float = 1.0):
    """Rows (h_coarse, difference, rate) of the table of `scheme`."""
    from . import api
    from ._lib import MpfcError
    finals, stats = {}, []
    for N in sizes:
        try:
            finals[N], st = final_state(N, scheme, omega=omega)
        except MpfcError as e:
            stats.append({"N": N, "error": str(e)})
            print(f"[convergence] scheme {scheme}, N = {N}: {e}", file=sys.stderr, flush=True)
            break
        stats.append(st)
        print(f"[convergence] scheme {scheme}, N = {N}: {st['steps']} steps in "
              f"{st['seconds']:.1f} s", file=sys.stderr, flush=True)
    done = [N for N in sizes if N in finals]
    rows = []
    for Nc, Nf in zip(done[:-1], done[1:]):
        d = (api.op_restrict(finals[Nf]) - finals[Nc]).cpu().numpy()
        diff = math.sqrt(float(np.mean(d * d)))
        rate = math.log2(rows[-1]["difference"] / diff) if rows else None
        rows.append({"h_coarse": 32.0 / Nc, "difference": diff, "rate": rate})
    return rows, stats


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--scheme", type=int, default=2, choices=(1, 2))
    ap.add_argument("--max-n", type=int, default=512)
    ap.add_argument("--omega", type=float, default=1.0,
                    help="relaxation factor of the smoother (below 1: V(2,2) on every grid)")
    a = ap.parse_args(argv)
    sizes = tuple(n for n in (32, 64, 128, 256, 512) if n <= a.max_n)
    rows, stats = table(a.scheme, sizes, omega=a.omega)
    print(json.dumps({"scheme": a.scheme, "rows": rows, "runs": stats}), flush=True)


if __name__ == "__main__":
    main()
