"""FP32-arithmetic precision study on the MeshBlock level set of 8 blocks of
128^3 (4 ghosts, 6th order, KO 0.5) tiling [-16, 16]^3: the conformally flat
star metric with matter blobs and U(-1e-6, 1e-6) noise, same-level neighbour
ghosts and frozen outer ghosts.

The same RK4 evolution (global dt = dx/4) runs once with FP64 arithmetic and
once with FP32 arithmetic (FP64 storage, stencil differences and Runge-Kutta
combination), each in its own autotuned launch shapes.  Reported: time per
step of each; at every checkpoint the L2
norms of the Hamiltonian and momentum constraints of each run and the L2 norm
of the difference of the two Hamiltonian-constraint fields; at the end, per
state field, the largest relative difference of the FP32 state from the FP64
state over interior points, relative to max(|u_64|, 1e-3 max|u_64|).

    python -m paper_2311_04989_amd.precision_study [--steps 100] [--every 10]

Prints progress to stderr and one JSON line to stdout.
"""
import argparse
import json
import math
import sys
import time

import numpy as np


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def evolve(bt, arith, steps, every, stream, h_ref=None):
    import torch

    from . import z4c as Z

    dev = "cuda:0"
    plan = Z.plan_for(bt, arith)
    frozen = torch.from_numpy(bt.frozen).to(dev)
    matter = torch.from_numpy(bt.matter).to(dev)
    regs = [torch.from_numpy(bt.u).to(dev)] + [torch.zeros_like(frozen) for _ in range(3)]
    cons = torch.zeros(bt.total_c, dtype=torch.float64, device=dev)
    norms = torch.zeros(len(bt.blocks) * 16, dtype=torch.float64, device=dev)
    plan.set_halo(Z.GHOST_NEIGHBOUR, frozen)
    plan.ghost_fill(Z.GHOST_NEIGHBOUR, regs[0], frozen, stream=stream)
    # launch shapes tuned for each arithmetic, so that the two runs compare
    # at their best (regs[1] and regs[3] are scratch until the first step)
    plan.autotune(regs[0], regs[1], regs[3], matter, reps=3, stream=stream)
    dv = bt.blocks[0].dx * bt.blocks[0].dy * bt.blocks[0].dz
    hslices = [slice(int(bt.coffsets[b]), int(bt.coffsets[b] + bt.field_stride[b]))
               for b in range(len(bt.blocks))]
    history, hfields = [], []

    def checkpoint(step):
        plan.constraints(regs[0], matter, cons, norms, stream=stream)
        n = norms.view(-1, 8, 2).sum(0).cpu().numpy()
        rec = {"step": step, "t": step * bt.dt, "H_L2": math.sqrt(n[0, 1]),
               "H_L1": float(n[0, 0]), "M_L2": math.sqrt(float(n[1:4, 1].sum())),
               "Theta_L2": math.sqrt(n[4, 1])}
        h = torch.cat([cons[s] for s in hslices])
        if h_ref is None:
            hfields.append(h.clone())
        else:
            rec["dH_L2"] = math.sqrt(float(((h - h_ref[len(history)]) ** 2).sum()) * dv)
        history.append(rec)
        log(f"[study] {'fp32' if arith else 'fp64'} step {step}: {rec}")

    checkpoint(0)
    ms = 0.0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    done = 0
    while done < steps:
        k = min(every, steps - done)
        e0.record(stream)
        for _ in range(k):
            r = plan.step(regs, matter, Z.RK4, bt.dt, Z.GHOST_NEIGHBOUR, frozen, stream=stream,
                          graph=True)
            assert r == 0
        e1.record(stream)
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
        done += k
        checkpoint(done)
    nonfinite = plan.check_finite(regs[0], stream=stream)
    final = regs[0].cpu().numpy()
    plan.close()
    return dict(ms_per_step=ms / steps, history=history, nonfinite=nonfinite), final, hfields


def field_errors(bt, g, o):
    from . import workloads as W

    out = {}
    for f in range(W.NF):
        oi = np.concatenate([bt.interior(o, b, f).ravel() for b in range(len(bt.blocks))])
        gi = np.concatenate([bt.interior(g, b, f).ravel() for b in range(len(bt.blocks))])
        scale = float(np.abs(oi).max())
        tau = 1e-3 * scale if scale > 0 else 1e-300
        d = np.abs(gi - oi)
        out[W.FIELDS[f]] = {"max_rel": float((d / np.maximum(np.abs(oi), tau)).max()),
                            "normwise": float(d.max() / scale) if scale > 0 else float(d.max()),
                            "max_abs_fp64": scale}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--n", type=int, default=128)
    args = ap.parse_args()
    import torch

    from . import workloads as W
    from . import z4c as Z

    assert torch.cuda.is_available(), "the precision study needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t0 = time.time()
    bt = W.config5(n=args.n)
    log(f"[study] generated {bt.name}: {bt.ninterior} interior points in {time.time() - t0:.1f}s")
    r64, u64, h64 = evolve(bt, Z.ARITH_FP64, args.steps, args.every, stream)
    r32, u32, _ = evolve(bt, Z.ARITH_FP32, args.steps, args.every, stream, h_ref=h64)
    del h64
    errs = field_errors(bt, u32, u64)
    worst = max(errs.items(), key=lambda kv: kv[1]["max_rel"])
    out = {"workload": f"8 MeshBlocks {args.n}^3 + 4 ghosts tiling [-16,16]^3, star metric + "
                       "matter blobs + 1e-6 noise, neighbour + frozen outer ghosts, 6th-order FD, "
                       f"KO 0.5, {args.steps} RK4 steps of dt = dx/4",
           "interior_points": bt.ninterior,
           "fp64": r64, "fp32": r32,
           "speedup_fp32": r64["ms_per_step"] / r32["ms_per_step"],
           "fp32_vs_fp64_final_state": errs,
           "worst_field": {"field": worst[0], **worst[1]}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
