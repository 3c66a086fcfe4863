"""Fixed-D sweeps to convergence and the two truncation-free extrapolations
on the GPU (the paper's Numerical benchmark procedure, on synthetic
integrals):

    python -m paper_2603_28648_amd.sweep_study --config cas22_22 --bond-dims 128,192,256,384,512

For every bond dimension: a fresh converged-like MPS of that D, full sweeps
until the energies of three subsequent sweeps agree within 1e-5 Ha, the
lowest energy and largest truncation error of the last sweep, and the time
spent in operator construction (dmrg_build_ops) and in the eigensolver.
Then the second-order fits of E against 1/D and against the truncation
error, each evaluated at zero.  One JSON line per bond dimension and a final
summary line on stdout; progress on stderr.
"""
import argparse
import json
import sys
import time

CONFIGS = {
    # name: (K, N, 2Sz, integral seed, MPS seed)
    "cas22_22": (22, 22, 0, 22, 1022),
    "cas10_10": (10, 10, 0, 10, 1010),
    "cas8_8": (8, 8, 0, 8, 1008),
}
# name: (ladder, residual refinement in the FP64 stage)
LADDERS = {"fp64": ((("fp64", None),), False),
           "mixed": ((("bf16x3", 1e-4), ("fp64", None)), False),
           "refined": ((("bf16x3", 1e-4), ("fp64", None)), True)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="cas22_22", choices=sorted(CONFIGS))
    ap.add_argument("--bond-dims", default="128,192,256,384,512")
    ap.add_argument("--sweep-tol", type=float, default=1e-5)
    ap.add_argument("--max-sweeps", type=int, default=8)
    ap.add_argument("--tol", type=float, default=1e-6, help="Davidson residual per window")
    ap.add_argument("--ladder", default="mixed", choices=sorted(LADDERS))
    ap.add_argument("--max-iter", type=int, default=100,
                    help="eigensolver iterations per window (residual refinement counts each inner "
                         "product); windows that stop short of --tol are counted in the output")
    args = ap.parse_args()

    import torch
    from synthetic import make_integrals, make_mps, mps_arrays, pack_psi
    from . import Context
    from .extrapolate import extrapolate_inverse_bond, extrapolate_truncation

    K, N, tsz, iseed, mseed = CONFIGS[args.config]
    h, eri = make_integrals(K, iseed)
    ds = [int(x) for x in args.bond_dims.split(",")]
    ctx = Context(0)
    E, eps = [], []

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    for D in ds:
        m = make_mps(K, N, tsz, D, 0, mseed)
        t0 = time.perf_counter()
        ctx.build_ops(0, h=h, eri=eri, n_elec=N, two_sz=tsz, mps_arrays=mps_arrays(m))
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t0
        psi = torch.from_numpy(pack_psi(m.bonds, 0, m.psi)).cuda()

        def sweep_log(msg, D=D):
            log(f"[sweeps] D={D} {msg}")

        t0 = time.perf_counter()
        ladder, refine = LADDERS[args.ladder]
        r = ctx.sweep_to_convergence(psi, D, sweep_tol=args.sweep_tol, max_sweeps=args.max_sweeps,
                                     tol=args.tol, ladder=ladder, log=sweep_log, refine=refine,
                                     max_iter=args.max_iter)
        wall = time.perf_counter() - t0
        sw = r["sweeps"]
        rec = {"bond_dim": D, "sweeps": len(sw), "converged": r["converged"], "energy": r["energy"],
               "max_trunc": r["max_trunc"], "energies": [s["min_energy"] for s in sw],
               "build_ops_s_per_sweep": sum(s["build_s"] for s in sw) / len(sw),
               "davidson_s_per_sweep": sum(s["davidson_s"] for s in sw) / len(sw),
               "initial_build_s": t_init, "wall_s": wall,
               "unconverged_windows": r["unconverged_windows"],
               "unconverged_per_sweep": [s["unconverged"] for s in sw]}
        print(json.dumps(rec), flush=True)
        log(f"[sweeps] D={D}: {len(sw)} sweeps, E={r['energy']:.10f}, eps={r['max_trunc']:.2e}, "
            f"converged={r['converged']}, {wall:.0f} s, windows not converged: {r['unconverged_windows']}")
        E.append(r["energy"])
        eps.append(r["max_trunc"])
    summary = {"config": args.config, "ladder": args.ladder, "bond_dims": ds, "energies": E,
               "max_trunc": eps}
    if len(ds) >= 3:
        summary["e_ext_inverse_bond"] = extrapolate_inverse_bond(ds, E)[0]
        summary["e_ext_truncation"] = extrapolate_truncation(eps, E)[0]
        summary["delta_e"] = summary["e_ext_inverse_bond"] - summary["e_ext_truncation"]
    print(json.dumps(summary), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
