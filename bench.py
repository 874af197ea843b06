"""Benchmark of the SoA/AoS particle-update hot path on one MI355X.

Timed step (the headline `value`): one pass of 50 RK2 steps in the ABC field
(A = B = C = 1, dt = 1e-3, periodic wrap) over 1e8 particles of the record
{int32 id; fp64 pos[3]; fp32 vel[3]} stored as SoA, inputs already resident
in HBM.  value = particle-updates/s = 1e8 * 50 * K / elapsed.

Every other row of the hot path is timed separately on the same GPU and
reported under "rows": the same RK2 workload in the LDS-staged and naive AoS
layouts, the Euler step at 1e8 particles in all layouts (the HBM headline),
the wide-record transposes and Euler-with-acceleration steps (3e7),
checkpointed RK2 forward and forward + adjoint (1e7, 200 steps, k = 20),
256 uneven sets stepped 100 times by one graph of persistent launches
versus one launch per set (tuned shape), removal of a seeded 1% of the
headline set by overwriting with the last particle, and fused array
expressions on the headline set (fused versus one launch per operation).
"copy" is the 16-byte copy kernel's bandwidth on 4 GiB, the achievable HBM
ceiling.  "fused_extra" is a labelled extra outside the benchmarked method:
every step of a job in one launch with the particles held in registers
(bit-identical results, one pass over memory per job instead of per step).

Prints ONE JSON line on stdout (progress goes to stderr).
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("particle-updates/s + achieved HBM GB/s (SoA vs AoS, fwd and fwd+adjoint), 1 GPU")
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_counters.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1710_03462_amd", "csrc", f)
                  for f in ("k_step.hip", "device_math.h", "trig.h", "launch.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_only(text):
    """Source text without comments and blank space: a comment edit leaves the
    compiled kernels, and so the counter data, valid."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "".join(text.split())


def sources_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p) as f:
            h.update(code_only(f.read()).encode())
    return h.hexdigest()[:16]


class Timer:
    """HIP events on torch's current stream, which every library call uses."""

    def __init__(self, torch):
        self.torch = torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.a.record()
        return self

    def __exit__(self, *exc):
        self.b.record()
        self.torch.cuda.synchronize()
        self.ms = self.a.elapsed_time(self.b)


def rate(count, ms):
    return count / (ms * 1e-3) if ms > 0 else float("nan")


def gbs(nbytes, ms):
    return nbytes / (ms * 1e-3) / 1e9 if ms > 0 else float("nan")


# ------------------------------------------------------------------- rows

def bench_rk2(torch, soax, ps, n, nsteps, layout, reps):
    ps.step(layout, "rk2_abc", 1e-3, nsteps, abc=[1, 1, 1], wrap=True)  # warm-up pass
    with Timer(torch) as t:
        for _ in range(reps):
            ps.step(layout, "rk2_abc", 1e-3, nsteps, abc=[1, 1, 1], wrap=True)
    per_launch = t.ms / (reps * nsteps)
    ups = rate(n * nsteps * reps, t.ms)
    phys = 60 if layout == "soa" else 2 * ps.stride
    return {"updates_per_s": ups, "ms_per_launch": per_launch,
            "alg_GBps": gbs(60 * n, per_launch), "physical_GBps": gbs(phys * n, per_launch),
            "steps": nsteps * reps}


def bench_integrators(torch, soax, ps, n, nsteps=10):
    """Heun and classical RK4 in the same field and symplectic Euler are not
    on the headline path; timed on the headline set in the SoA and LDS-staged
    AoS layouts (60 B per particle-step algorithmic for the field integrators,
    as for RK2)."""
    out = {}
    for integ in ("heun_abc", "rk4_abc"):
        for lay in ("soa", "aos"):
            ps.step(lay, integ, 1e-3, 1, abc=[1, 1, 1], wrap=True)
            with Timer(torch) as t:
                ps.step(lay, integ, 1e-3, nsteps, abc=[1, 1, 1], wrap=True)
            per = t.ms / nsteps
            out[f"{integ}_{lay}"] = {"updates_per_s": rate(n * nsteps, t.ms), "ms_per_launch": per,
                                     "alg_GBps": gbs(60 * n, per)}
    return out


def bench_fused(torch, soax, si, ps, n, nsteps, stepwise_ms):
    """A labelled extra, not the benchmarked method (which passes over every
    array at each step): nsteps steps in one launch with every particle held
    in registers (soax_step_fused, bit-identical to the separate steps), on
    the headline set (RK2, and Euler) and on the 1e5-particle Euler workload.
    Bound by fp64 arithmetic instead of HBM; the arrays move once per job."""
    out = {}
    for integ, abc in (("rk2_abc", [1, 1, 1]), ("euler", None)):
        ps.step_fused(integ, 1e-3, 2, abc=abc, wrap=True)
        with Timer(torch) as t:
            ps.step_fused(integ, 1e-3, nsteps, abc=abc, wrap=True)
        out[f"{integ}_1e8"] = {"nsteps": nsteps, "ms": t.ms, "updates_per_s": rate(n * nsteps, t.ms)}
    out["rk2_abc_1e8"]["over_stepwise"] = stepwise_ms / out["rk2_abc_1e8"]["ms"]
    small_n, small_steps = 100_000, 100
    small = soax.ParticleSet(si.BASE_FIELDS, small_n, aos=False)
    small.fill(seed=0)
    small.step_fused("euler", 1e-3, small_steps, wrap=True)
    with Timer(torch) as t:
        small.step_fused("euler", 1e-3, small_steps, wrap=True)
    out["euler_1e5"] = {"nsteps": small_steps, "ms": t.ms,
                        "updates_per_s": rate(small_n * small_steps, t.ms)}
    small.close()
    return out


def bench_aosoa(torch, soax, si, n, nsteps=20):
    """The tiled (AoSoA, 64-particle tiles) copy of the headline set: Euler and
    RK2 steps timed like the SoA rows (60 B per particle-step algorithmic)."""
    ps = soax.ParticleSet(si.BASE_FIELDS, n, aos=False, aosoa=True)
    ps.fill(seed=0, vel_mode=1, abc=[1, 1, 1])
    ps.soa_to_aosoa()
    out = {}
    for integ, steps in (("euler", nsteps), ("rk2_abc", nsteps)):
        ps.step("aosoa", integ, 1e-3, 2, abc=[1, 1, 1], wrap=True)
        with Timer(torch) as t:
            ps.step("aosoa", integ, 1e-3, steps, abc=[1, 1, 1], wrap=True)
        per = t.ms / steps
        out[integ] = {"updates_per_s": rate(n * steps, t.ms), "ms_per_launch": per,
                      "alg_GBps": gbs(60 * n, per)}
    with Timer(torch) as t:
        ps.soa_to_aosoa()
    out["soa_to_aosoa"] = {"ms": t.ms, "GBps": gbs(2 * ps.soa_bytes * n, t.ms)}
    ps.close()
    torch.cuda.empty_cache()
    return out


def bench_euler(torch, soax, ps, n, nsteps, layout):
    ps.step(layout, "euler", 1e-3, 2, wrap=True)
    with Timer(torch) as t:
        ps.step(layout, "euler", 1e-3, nsteps, wrap=True)
    per_launch = t.ms / nsteps
    phys = 60 if layout == "soa" else 2 * ps.stride
    return {"updates_per_s": rate(n * nsteps, t.ms), "ms_per_launch": per_launch,
            "alg_GBps": gbs(60 * n, per_launch), "physical_GBps": gbs(phys * n, per_launch),
            "frac_of_peak": gbs(phys * n, per_launch) / HBM_PEAK_GBS, "steps": nsteps}


def bench_small_euler(torch, soax, si, n=100_000, nsteps=100):
    """The 1e5-particle Euler workload: 4 MB of state, cache-resident and
    launch-bound, reported as updates/s in every layout, with one launch per
    step and with the steps replayed from a captured graph."""
    ps = soax.ParticleSet(si.BASE_FIELDS, n)
    ps.fill(seed=0)
    ps.soa_to_aos()
    out = {"n": n, "nsteps": nsteps}
    for lay in ("soa", "aos", "aos_naive"):
        ps.step(lay, "euler", 1e-3, 10, wrap=True)
        with Timer(torch) as t:
            ps.step(lay, "euler", 1e-3, nsteps, wrap=True)
        # wall time around single-step C-ABI calls: host cost per call, and
        # call + completion
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            ps.step(lay, "euler", 1e-3, 1, wrap=True)
        t1 = time.perf_counter()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        # the same steps captured once into a graph and replayed
        g = ps.step_graph(lay, "euler", 1e-3, nsteps, wrap=True)
        g.launch()
        with Timer(torch) as tg:
            for _ in range(5):
                g.launch()
        g.close()
        out[lay] = {"updates_per_s": rate(n * nsteps, t.ms), "us_per_step": t.ms * 1e3 / nsteps,
                    "call_us": (t1 - t0) * 1e6 / nsteps,
                    "wall_us_per_step": (t2 - t0) * 1e6 / nsteps,
                    "graph_us_per_step": tg.ms * 1e3 / (5 * nsteps),
                    "graph_updates_per_s": rate(5 * n * nsteps, tg.ms)}
    ps.close()
    return out


def bench_copy(torch, soax, nbytes=4 << 30):
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    soax.copy(dst, src)
    reps = 10
    with Timer(torch) as t:
        for _ in range(reps):
            soax.copy(dst, src)
    per = t.ms / reps
    out = {"bytes": nbytes, "ms_per_launch": per, "GBps": gbs(2 * nbytes, per),
           "frac_of_peak": gbs(2 * nbytes, per) / HBM_PEAK_GBS}
    del src, dst
    return out


def bench_probes(torch, soax, n, reps=20):
    """The memory patterns of the streaming SoA steps with no arithmetic
    (soax_probe), on arrays allocated like a ParticleSet's (one tensor per
    array): the ceiling each step kernel is measured against.  rk2 and euler
    move 60 B per particle, read 24 B, write 36 B."""
    pos = [torch.rand(n, dtype=torch.float64, device="cuda") * 6.0 for _ in range(3)]
    vel = [torch.randn(n, dtype=torch.float32, device="cuda") for _ in range(3)]
    out = {"n": n}
    for pat, nbytes in (("rk2", 60), ("euler", 60), ("read", 24), ("write", 36)):
        for _ in range(2):
            soax.probe(pat, pos, vel)
        with Timer(torch) as t:
            for _ in range(reps):
                soax.probe(pat, pos, vel)
        per = t.ms / reps
        out[pat] = {"bytes_per_particle": nbytes, "ms_per_launch": per,
                    "GBps": gbs(nbytes * n, per), "frac_of_peak": gbs(nbytes * n, per) / HBM_PEAK_GBS}
    del pos, vel
    torch.cuda.empty_cache()
    return out


def bench_expr_euler(torch, soax, si, ns=(100_000, 100_000_000), nsteps=20, dt=1e-3):
    """The library's generated form of the Euler update against the
    hand-written SoA step, call overhead included (the comparison of
    Section 4.2.2): per step, pos_d = pos_d + dt * vel_d as three fused
    expression launches, or one soax_step launch (no wrap: the expressions
    have none).  Kernel time from events, wall time around the calls."""
    out = {}
    for n in ns:
        ps = soax.ParticleSet(si.BASE_FIELDS, n, aos=False)
        ps.fill(seed=0)
        progs = [ps.arr("pos", d) + dt * ps.arr("vel", d) for d in range(3)]

        def generated():
            for d in range(3):
                ps.assign(("pos", d), progs[d])

        def hand_written():
            ps.step("soa", "euler", dt, 1, wrap=False)

        row = {"nsteps": nsteps}
        for name, fn in (("generated", generated), ("hand_written", hand_written)):
            for _ in range(3):
                fn()
            with Timer(torch) as t:
                w0 = time.perf_counter()
                for _ in range(nsteps):
                    fn()
                torch.cuda.synchronize()
                w1 = time.perf_counter()
            row[name] = {"kernel_ms_per_step": t.ms / nsteps,
                         "wall_ms_per_step": (w1 - w0) * 1e3 / nsteps,
                         "alg_GBps": gbs(60 * n, t.ms / nsteps)}
        row["generated_over_hand_written_wall"] = (row["generated"]["wall_ms_per_step"] /
                                                   row["hand_written"]["wall_ms_per_step"])
        row["generated_over_hand_written_kernel"] = (row["generated"]["kernel_ms_per_step"] /
                                                     row["hand_written"]["kernel_ms_per_step"])
        out[f"n={n:.0e}"] = row
        ps.close()
        torch.cuda.empty_cache()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_wide(torch, soax, si, n):
    ps = soax.ParticleSet(si.WIDE_FIELDS, n)
    ps.fill(seed=0)
    ps.soa_to_aos()
    ps.aos_to_soa()
    ps.step("soa", "euler_acc", 1e-3, 2, wrap=True)
    alg_x = 2 * ps.soa_bytes
    phys_x = ps.soa_bytes + ps.stride
    with Timer(torch) as t1:
        ps.aos_to_soa()
    with Timer(torch) as t2:
        ps.step("soa", "euler_acc", 1e-3, 20, wrap=True)
    with Timer(torch) as t3:
        ps.soa_to_aos()
    res = {"n": n, "aos_to_soa": {"ms": t1.ms, "alg_GBps": gbs(alg_x * n, t1.ms),
                                  "physical_GBps": gbs(phys_x * n, t1.ms)},
           "euler_acc_soa": {"updates_per_s": rate(n * 20, t2.ms), "ms_per_launch": t2.ms / 20,
                             "alg_GBps": gbs(84 * n, t2.ms / 20)},
           "soa_to_aos": {"ms": t3.ms, "alg_GBps": gbs(alg_x * n, t3.ms),
                          "physical_GBps": gbs(phys_x * n, t3.ms)}}
    ps.close()
    return res


def bench_remove(torch, soax, si, n, frac=0.01, reps=3):
    """Removal by overwriting with the last particle on both copies of the
    headline set: a seeded 1% of the particles flagged.  Each repetition
    first regrows the set to n (untimed)."""
    ps = soax.ParticleSet(si.BASE_FIELDS, n)
    ps.fill(seed=0, vel_mode=1, abc=[1, 1, 1])
    ps.soa_to_aos()
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    flags = (torch.rand(n, generator=g, device="cuda") < frac).to(torch.uint8)
    m = int(flags.sum())
    n_new = n - m
    moves = int(flags[:n_new].sum())  # flagged slots below the new size
    times = []
    for _ in range(reps + 1):
        ps.resize(n)
        with Timer(torch) as t:
            got = ps.remove_flagged(flags)
        assert got == n_new
        times.append(t.ms)
    ms = min(times[1:])
    # algorithmic bytes: every flag read once; every moved particle read and
    # written in both copies (40 B SoA + 48 B AoS record)
    alg = n + moves * 2 * (ps.soa_bytes + ps.stride)
    out = {"n": n, "removed": m, "moves": moves, "ms": ms, "alg_GBps": gbs(alg, ms),
           "particles_per_s": rate(n, ms)}
    ps.close()
    del flags
    return out


def _unfused(torch, soax, E, dst, expr):
    """Evaluate a program one operation per launch, temporaries in HBM (the
    separate loops the fused kernel replaces)."""
    stack = []
    steps = expr.steps
    for pos, (op, key, value) in enumerate(steps):
        if op in (E.ARRAY, E.CONST):
            stack.append(E.Expr([(op, key, value)]))
            continue
        last = pos == len(steps) - 1
        if op in (E.NEG, E.ABS, E.SQRT):
            x = stack.pop()
            node = E.Expr(x.steps + [(op, None, 0.0)])
        else:
            b = stack.pop()
            a = stack.pop()
            node = E.Expr(a.steps + b.steps + [(op, None, 0.0)])
        out = dst if last else torch.empty(dst.numel(), dtype=torch.float64, device="cuda")
        soax.evaluate(out, node)
        stack.append(E.array(out))


def bench_expr(torch, soax, si, n, reps=5):
    """Fused array expressions on the headline set: the paper's example
    pos_0 = vel_1 - vel_2 (16 B per particle), and
    pos_0 = pos_0 + dt * sqrt(vel_0^2 + vel_1^2 + vel_2^2) fused (28 B) versus
    one launch per operation with double temporaries."""
    from paper_1710_03462_amd import expr as E
    ps = soax.ParticleSet(si.BASE_FIELDS, n, aos=False)
    ps.fill(seed=0)
    x = ps.array("pos", 0)
    vx, vy, vz = (ps.array("vel", d) for d in range(3))
    diff = ps.arr("vel", 1) - ps.arr("vel", 2)
    ps.assign(("pos", 0), diff)  # compiles
    with Timer(torch) as t1:
        for _ in range(reps):
            ps.assign(("pos", 0), diff)
    ms_diff = t1.ms / reps
    speed = E.sqrt(E.array(vx) * E.array(vx) + E.array(vy) * E.array(vy) +
                   E.array(vz) * E.array(vz))
    prog = E.array(x) + 1e-3 * speed
    soax.evaluate(x, prog)
    _unfused(torch, soax, E, x, prog)
    with Timer(torch) as t2:
        for _ in range(reps):
            soax.evaluate(x, prog)
    with Timer(torch) as t3:
        for _ in range(reps):
            _unfused(torch, soax, E, x, prog)
    fused, unfused = t2.ms / reps, t3.ms / reps
    ops = sum(1 for op, _, _ in prog.steps if op not in (E.ARRAY, E.CONST))
    out = {"n": n,
           "paper_example": {"expr": "pos0 = vel1 - vel2", "ms": ms_diff,
                             "alg_GBps": gbs(16 * n, ms_diff)},
           "fused": {"expr": "pos0 = pos0 + dt*sqrt(vx^2+vy^2+vz^2)", "ms": fused,
                     "alg_GBps": gbs(28 * n, fused)},
           "unfused": {"launches": ops, "ms": unfused},
           "fusion_speedup": unfused / fused}
    ps.close()
    torch.cuda.empty_cache()
    return out


def bench_adjoint(torch, soax, si, n, nsteps=200, k=20):
    src = soax.ParticleSet(si.BASE_FIELDS, n, aos=False)
    src.fill(seed=0)
    x0 = torch.stack([src.array("pos", d) for d in range(3)]).contiguous()
    src.fill(seed=1)
    target = torch.stack([src.array("pos", d) for d in range(3)]).contiguous()
    src.close()
    abc = soax.autograd._host3(torch.tensor([1.0, 0.8, 0.6], dtype=torch.float64))
    dt = 5e-3
    soax.forward_ckpt(x0, abc, dt, nsteps, k)
    with Timer(torch) as tf:
        xT, tape = soax.forward_ckpt(x0, abc, dt, nsteps, k)
    with Timer(torch) as tb:
        xT, tape = soax.forward_ckpt(x0, abc, dt, nsteps, k)
        loss, lam = soax.sqdist_loss(xT, target)
        gx, gabc = soax.adjoint(tape, lam, abc, dt, nsteps, k)
    res = {"n": n, "nsteps": nsteps, "k": k,
           "fwd": {"ms": tf.ms, "particle_steps_per_s": rate(n * nsteps, tf.ms)},
           "fwd_adjoint": {"ms": tb.ms, "particle_steps_per_s": rate(n * nsteps, tb.ms)},
           "loss": float(loss.item())}
    del xT, tape, lam, gx
    # the same with the positions kept inside 48-byte AoS records (pos at byte 8)
    from paper_1710_03462_amd import autograd as A
    stride, off = 48, 8
    rec = torch.zeros((n, stride), dtype=torch.uint8, device="cuda")
    rec[:, off:off + 24] = x0.t().contiguous().view(torch.uint8).view(n, 24)
    rec = rec.view(-1)
    out = torch.empty_like(rec)
    lam_rec = torch.empty_like(rec)
    gx_rec = torch.empty_like(rec)
    A.forward_ckpt_records(rec, out, off, stride, n, abc, dt, nsteps, k)
    with Timer(torch) as taf:
        tape = A.forward_ckpt_records(rec, out, off, stride, n, abc, dt, nsteps, k)
    del tape
    with Timer(torch) as tab:
        tape = A.forward_ckpt_records(rec, out, off, stride, n, abc, dt, nsteps, k)
        loss_a = A.sqdist_loss_records(out, target, lam_rec, off, stride, n)
        A.adjoint_records(tape, lam_rec, gx_rec, off, stride, n, abc, dt, nsteps, k)
    res["fwd_aos"] = {"ms": taf.ms, "particle_steps_per_s": rate(n * nsteps, taf.ms)}
    res["fwd_adjoint_aos"] = {"ms": tab.ms, "particle_steps_per_s": rate(n * nsteps, tab.ms)}
    res["soa_over_aos_fwd"] = taf.ms / tf.ms
    res["soa_over_aos_fwd_adjoint"] = tab.ms / tb.ms
    res["aos_loss_equal"] = bool(float(loss_a.item()) == res["loss"])
    del x0, target, rec, out, lam_rec, gx_rec, tape
    return res


def bench_batch(torch, soax, si, nsets=256, nsteps=100):
    sizes, dts, abc = si.batch_plan(nsets, seed=0)
    sets = []
    for s, n in enumerate(sizes):
        ps = soax.ParticleSet(si.BASE_FIELDS, int(n), aos=False)
        ps.fill(seed=s, vel_mode=1, abc=abc[s])
        sets.append(ps)
    total = int(sizes.sum())
    b = soax.Batch(sets)
    b.step(dts, abc, 1, mode=soax.PERSISTENT)  # the tuner times the last step's dt and amplitudes
    t0 = time.perf_counter()
    cfg = b.tune()
    tune_s = time.perf_counter() - t0
    b.step(dts, abc, nsteps, mode=soax.GRAPH)  # capture + warm-up
    with Timer(torch) as tg:
        b.step(dts, abc, nsteps, mode=soax.GRAPH)
    with Timer(torch) as tp:
        b.step(dts, abc, nsteps, mode=soax.PERSISTENT)
    b.step(dts, abc, 2, mode=soax.PER_SET)
    with Timer(torch) as ts:
        b.step(dts, abc, nsteps, mode=soax.PER_SET)
    res = {"nsets": nsets, "particles": total, "nsteps": nsteps,
           "tuned": {"block": cfg[0], "per_thread": cfg[1], "blocks_per_cu": cfg[2],
                     "tune_s": tune_s},
           "graph": {"ms": tg.ms, "updates_per_s": rate(total * nsteps, tg.ms),
                     "alg_GBps": gbs(60 * total * nsteps, tg.ms)},
           "persistent_eager": {"ms": tp.ms, "updates_per_s": rate(total * nsteps, tp.ms)},
           "per_set_launches": {"ms": ts.ms, "updates_per_s": rate(total * nsteps, ts.ms),
                                "launches": nsets * nsteps},
           "graph_speedup_vs_per_set": ts.ms / tg.ms}
    b.close()
    for ps in sets:
        ps.close()
    return res


SWEEP_LAYOUTS = ("soa", "aos", "aos_naive")
SWEEP_WARM = 5


def sweep_steps(n, steps=None):
    """Timed steps of one sweep point: 2e8 particle-steps, 20 to 2000 steps."""
    return steps if steps else max(20, min(2000, int(2e8 // n)))


def bench_sweep(torch, soax, si, sizes=(0, 4, 8, 16, 32),
                ns=(1_000, 10_000, 100_000, 1_000_000, 10_000_000, 100_000_000), steps=None):
    """The paper's GPU experiment (Section 3.2) on this GPU: the Euler step of
    Listing 4's particle (float x[3], v[3], temp[SIZE]) in SoA, LDS-staged AoS
    and per-thread AoS (the paper's access pattern), time per particle-step
    against the particle count N.  Algorithmic bytes per particle-step: 36
    (x and v read, x written); the AoS copies move whole records (2 * stride).
    Per point and layout: SWEEP_WARM untimed steps, then sweep_steps() timed
    ones, each one launch; --sweep-report reads the same sequence of launches
    back from a rocprofv3 trace."""
    rows = []
    for size in sizes:
        fields = si.particle_size_fields(size)
        for n in ns:
            ps = soax.ParticleSet(fields, n)
            ps.fill(seed=0)
            ps.soa_to_aos()
            nsteps = sweep_steps(n, steps)
            row = {"SIZE": size, "N": n, "record_bytes": ps.stride, "nsteps": nsteps}
            for lay in SWEEP_LAYOUTS:
                ps.step(lay, "euler", 1e-3, SWEEP_WARM, wrap=False)
                with Timer(torch) as t:
                    ps.step(lay, "euler", 1e-3, nsteps, wrap=False)
                per = t.ms / nsteps
                row[lay] = {"ns_per_particle": per * 1e6 / n,
                            "alg_GBps": gbs(36 * n, per),
                            "physical_GBps": gbs((36 if lay == "soa" else 2 * ps.stride) * n, per)}
            row["aos_over_soa"] = row["aos"]["ns_per_particle"] / row["soa"]["ns_per_particle"]
            row["naive_over_soa"] = (row["aos_naive"]["ns_per_particle"] /
                                     row["soa"]["ns_per_particle"])
            log(f"[sweep] SIZE={size:2d} N={n:>9d}  soa {row['soa']['ns_per_particle']:.4f} ns  "
                f"aos {row['aos']['ns_per_particle']:.4f}  naive "
                f"{row['aos_naive']['ns_per_particle']:.4f}")
            rows.append(row)
            ps.close()
            del ps
            torch.cuda.empty_cache()
    return rows


SWEEP_KERNELS = {"soa": re.compile(r"(?<![A-Za-z_])soa_step_kernel<"),
                 "aos": re.compile(r"(?<![A-Za-z_])aos_step_kernel<"),
                 "aos_naive": re.compile(r"(?<![A-Za-z_])aos_naive_kernel<")}


def _find_csv(path, suffix):
    if os.path.isfile(path):
        return path if path.endswith(suffix) else None
    for dirpath, _, files in os.walk(path):
        for f in sorted(files):
            if f.endswith(suffix):
                return os.path.join(dirpath, f)
    return None


def _col(row, *names):
    for nm in names:
        if nm in row and row[nm] != "":
            return row[nm]
    raise KeyError(names)


def sweep_report(trace_dir, sizes, ns, steps=None):
    """Per-launch kernel durations (and counters, when the directory holds a
    counter run) of the sweep, read from rocprofv3 output: the way the paper
    times its GPU experiment, with each kernel's execution isolated from the
    host's launch overhead (Section 3.2).  The step launches are matched, in
    dispatch order, to the sweep's sequence of points and layouts; every
    matched run must hold SWEEP_WARM + nsteps launches of the layout's kernel.
    Time per particle-step is the median duration of the timed launches / N."""
    import csv
    import statistics
    plan = [(size, n, lay, sweep_steps(n, steps)) for size in sizes for n in ns
            for lay in SWEEP_LAYOUTS]

    def runs_of(dispatches):
        # dispatches: (id, layout, grid, payload) in dispatch order
        runs = []
        for d in dispatches:
            if runs and runs[-1]["layout"] == d[1] and runs[-1]["grid"] == d[2]:
                runs[-1]["items"].append(d[3])
            else:
                runs.append({"layout": d[1], "grid": d[2], "items": [d[3]]})
        return runs

    def layout_of(name):
        for lay, rx in SWEEP_KERNELS.items():
            if rx.search(name):
                return lay
        return None

    def check(runs, what):
        if len(runs) != len(plan):
            raise SystemExit(f"{what}: {len(runs)} runs of step launches, the sweep has "
                             f"{len(plan)} points x layouts")
        for r, (size, n, lay, nst) in zip(runs, plan):
            if r["layout"] != lay or len(r["items"]) != SWEEP_WARM + nst:
                raise SystemExit(f"{what}: run {r['layout']} x{len(r['items'])} does not match "
                                 f"SIZE={size} N={n} {lay} ({SWEEP_WARM}+{nst} launches)")

    out = {}
    trace = _find_csv(trace_dir, "kernel_trace.csv")
    if trace:
        disp = []
        with open(trace) as f:
            for row in csv.DictReader(f):
                lay = layout_of(row["Kernel_Name"])
                if lay is None:
                    continue
                dur = int(_col(row, "End_Timestamp")) - int(_col(row, "Start_Timestamp"))
                disp.append((int(_col(row, "Dispatch_Id")), lay,
                             int(_col(row, "Grid_Size_X", "Grid_Size")), dur))
        disp.sort()
        runs = runs_of(disp)
        check(runs, trace)
        for r, (size, n, lay, nst) in zip(runs, plan):
            ns_med = statistics.median(r["items"][SWEEP_WARM:])
            out.setdefault((size, n), {})[lay] = {"kernel_ns": ns_med,
                                                 "ns_per_particle": ns_med / n,
                                                 "SoA_alg_GBps": 36 * n / ns_med}
    cnt = _find_csv(trace_dir, "counter_collection.csv")
    if cnt:
        per = {}
        with open(cnt) as f:
            for row in csv.DictReader(f):
                lay = layout_of(row["Kernel_Name"])
                if lay is None:
                    continue
                key = (int(_col(row, "Dispatch_Id")), lay, int(_col(row, "Grid_Size_X", "Grid_Size")))
                per.setdefault(key, {})
                nm = row["Counter_Name"]
                per[key][nm] = per[key].get(nm, 0.0) + float(row["Counter_Value"])
        disp = sorted((k[0], k[1], k[2], v) for k, v in per.items())
        runs = runs_of(disp)
        check(runs, cnt)
        for r, (size, n, lay, nst) in zip(runs, plan):
            timed = r["items"][SWEEP_WARM:]
            names = sorted(timed[0])
            avg = {nm: sum(t.get(nm, 0.0) for t in timed) / len(timed) for nm in names}
            out.setdefault((size, n), {}).setdefault(lay, {})["counters_per_launch"] = avg
    if not out:
        raise SystemExit(f"no kernel_trace.csv or counter_collection.csv under {trace_dir}")
    return out


def sweep_report_rows(dirs, sizes, ns, steps=None):
    """sweep_report over several rocprofv3 output directories of the same
    sweep (a kernel trace and counter runs), merged per point and layout."""
    out = {}
    for d in dirs:
        for key, lays in sweep_report(d, sizes, ns, steps).items():
            for lay, v in lays.items():
                tgt = out.setdefault(key, {}).setdefault(lay, {})
                cnt = v.pop("counters_per_launch", None)
                tgt.update(v)
                if cnt:
                    tgt.setdefault("counters_per_launch", {}).update(cnt)
    rows = []
    for (size, n), v in sorted(out.items()):
        row = {"SIZE": size, "N": n, **v}
        if all("ns_per_particle" in v.get(lay, {}) for lay in SWEEP_LAYOUTS):
            row["aos_over_soa"] = v["aos"]["ns_per_particle"] / v["soa"]["ns_per_particle"]
            row["naive_over_soa"] = v["aos_naive"]["ns_per_particle"] / v["soa"]["ns_per_particle"]
        rows.append(row)
    return rows


def sweep_markdown(rows):
    """The merged sweep rows as a markdown table: kernel time per launch,
    time per particle-step, the AoS/SoA ratios and, where counters were
    taken, the L2 hit rate TCC_HIT / (TCC_HIT + TCC_MISS) and the vector-L1
    hit rate 1 - (TCP_TCC_READ_REQ + TCP_TCC_WRITE_REQ) /
    TCP_TOTAL_CACHE_ACCESSES."""
    def hits(v):
        c = v.get("counters_per_launch", {})
        l2 = l1 = ""
        if c.get("TCC_HIT_sum", 0) + c.get("TCC_MISS_sum", 0) > 0:
            l2 = f"{c['TCC_HIT_sum'] / (c['TCC_HIT_sum'] + c['TCC_MISS_sum']):.2f}"
        if c.get("TCP_TOTAL_CACHE_ACCESSES_sum", 0) > 0:
            miss = c.get("TCP_TCC_READ_REQ_sum", 0) + c.get("TCP_TCC_WRITE_REQ_sum", 0)
            l1 = f"{1 - miss / c['TCP_TOTAL_CACHE_ACCESSES_sum']:.2f}"
        return l1, l2

    def traffic(v, n):
        # bytes past the L2 per particle-step, FETCH_SIZE and WRITE_SIZE (KiB
        # per dispatch) scaled by the copy-kernel calibration of the committed
        # counter data (FETCH_SIZE counts half the bytes on this GPU)
        c = v.get("counters_per_launch", {})
        if "FETCH_SIZE" not in c and "WRITE_SIZE" not in c:
            return ""
        try:
            with open(PROFILE_TRAFFIC) as f:
                cal = json.load(f)["calibration"]
        except (OSError, ValueError, KeyError):
            cal = {"read_factor": 1.0, "write_factor": 1.0}
        rd = c.get("FETCH_SIZE", 0.0) * 1024 * cal["read_factor"] / n
        wr = c.get("WRITE_SIZE", 0.0) * 1024 * cal["write_factor"] / n
        return f"{rd:.1f}+{wr:.1f}"

    with_traffic = any("FETCH_SIZE" in r.get(lay, {}).get("counters_per_launch", {})
                       or "WRITE_SIZE" in r.get(lay, {}).get("counters_per_launch", {})
                       for r in rows for lay in SWEEP_LAYOUTS)
    head = ("| SIZE | N | SoA µs | AoS µs | naive µs | SoA ns/p | AoS/SoA | naive/SoA | "
            "L1 hit soa/aos/naive | L2 hit soa/aos/naive |")
    rule = "|---|---|---|---|---|---|---|---|---|---|"
    if with_traffic:
        head += " read+write B/particle soa / aos / naive |"
        rule += "---|"
    lines = [head, rule]
    for r in rows:
        us = [f"{r[lay]['kernel_ns'] / 1e3:.2f}" if "kernel_ns" in r.get(lay, {}) else ""
              for lay in SWEEP_LAYOUTS]
        nsp = f"{r['soa']['ns_per_particle']:.4f}" if "ns_per_particle" in r.get("soa", {}) else ""
        ratio = [f"{r[k]:.2f}" if k in r else "" for k in ("aos_over_soa", "naive_over_soa")]
        h = [hits(r.get(lay, {})) for lay in SWEEP_LAYOUTS]
        line = (f"| {r['SIZE']} | {r['N']:.0e} | {' | '.join(us)} | {nsp} | "
                f"{' | '.join(ratio)} | {'/'.join(x[0] for x in h)} | "
                f"{'/'.join(x[1] for x in h)} |")
        if with_traffic:
            line += f" {' / '.join(traffic(r.get(lay, {}), r['N']) for lay in SWEEP_LAYOUTS)} |"
        lines.append(line)
    return "\n".join(lines)


def cpu_baseline(ref, si, target_s=14.0):
    """The oracle's RK2 step on a bounded sample of the headline workload, in
    SoA (the reported value) and, on half as many particles, in AoS records
    (the CPU's SoA/AoS ratio beside the GPU's).  The sample is sized from a
    short probe, which overestimates the cost per update about twofold, so the
    timed SoA run lands near 7-10 s and the AoS run near half that."""
    sch = ref.Schema(si.BASE_FIELDS)
    cores = ref.threads()
    probe_n, probe_steps = 20000, 5
    arrays = ref.fill(sch, probe_n, seed=0, vel_mode=1, abc=[1, 1, 1])
    t0 = time.perf_counter()
    ref.step_soa(sch, arrays, ref.RK2_ABC, 1e-3, probe_steps, abc=[1, 1, 1], wrap=True)
    probe = (time.perf_counter() - t0) / (probe_n * probe_steps)
    n = int(min(1e8, max(1e4, target_s / probe / 50)))
    arrays = ref.fill(sch, n, seed=0, vel_mode=1, abc=[1, 1, 1])
    t0 = time.perf_counter()
    ref.step_soa(sch, arrays, ref.RK2_ABC, 1e-3, 50, abc=[1, 1, 1], wrap=True)
    el = time.perf_counter() - t0
    del arrays
    n_aos = n // 2
    aos = ref.soa_to_aos(sch, ref.fill(sch, n_aos, seed=0, vel_mode=1, abc=[1, 1, 1]))
    t0 = time.perf_counter()
    ref.step_aos(sch, aos, n_aos, ref.RK2_ABC, 1e-3, 50, abc=[1, 1, 1], wrap=True)
    el_aos = time.perf_counter() - t0
    soa_rate, aos_rate = n * 50 / el, n_aos * 50 / el_aos
    return {"value": soa_rate, "unit": "particle-updates/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "aos_value": aos_rate, "soa_over_aos": soa_rate / aos_rate,
            "sample": f"{n} particles x 50 RK2 steps of the same record and field "
                      f"(SoA, OpenMP static schedule), {el:.1f} s; AoS records: {n_aos} "
                      f"particles x 50 steps, {el_aos:.1f} s"}


def traffic_from_profiles(kernel, launches_bytes_key):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None when
    the kernel sources changed since the counters were taken."""
    try:
        with open(PROFILE_TRAFFIC) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    if data.get("sources_sha256_16") != sources_hash():
        return None
    ent = data.get("kernels", {}).get(kernel)
    return ent.get(launches_bytes_key) if ent else None


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed 50-step passes")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=float, default=1e8, help="particles of the headline workload")
    ap.add_argument("--rows", default="all",
                    help="comma list of extra rows: aos,euler,small,copy,probes,wide,adjoint,"
                         "batch,remove,expr,expr_euler,integrators,aosoa,fused | all | none")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--sweep", action="store_true",
                    help="run only the N x SIZE sweep of the paper's GPU experiment and print "
                         "its rows as one JSON line")
    ap.add_argument("--sweep-sizes", default="0,4,8,16,32")
    ap.add_argument("--sweep-ns", default="1e3,1e4,1e5,1e6,1e7,1e8")
    ap.add_argument("--sweep-steps", type=int, default=0,
                    help="timed steps per sweep point (default: 2e8 particle-steps, 20..2000)")
    ap.add_argument("--sweep-report", metavar="DIR[,DIR...]",
                    help="no GPU work: read the rocprofv3 kernel trace and/or counters of "
                         "--sweep runs (same sizes, ns and steps) from each DIR and print "
                         "per-launch kernel times and counters as one JSON line")
    ap.add_argument("--md", action="store_true",
                    help="with --sweep-report: print a markdown table instead")
    args = ap.parse_args()
    if args.sweep_report:
        sizes = tuple(int(x) for x in args.sweep_sizes.split(","))
        ns = tuple(int(float(x)) for x in args.sweep_ns.split(","))
        rows = sweep_report_rows(args.sweep_report.split(","), sizes, ns, args.sweep_steps or None)
        print(sweep_markdown(rows) if args.md else json.dumps({"sweep_report": rows}), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard by particle range with no communication; one GPU is measured)",
              file=sys.stderr)
        return 2

    import torch

    import paper_1710_03462_amd as soax
    import synth_inputs as si

    soax.lib()
    torch.cuda.set_device(0)
    if args.sweep:
        sizes = tuple(int(x) for x in args.sweep_sizes.split(","))
        ns = tuple(int(float(x)) for x in args.sweep_ns.split(","))
        print(json.dumps({"sweep": bench_sweep(torch, soax, si, sizes, ns,
                                               args.sweep_steps or None),
                          "device": torch.cuda.get_device_name(0)}), flush=True)
        return 0
    rows = {"aos", "euler", "small", "copy", "probes", "wide", "adjoint", "batch", "remove",
            "expr", "expr_euler", "integrators", "aosoa", "fused"} \
        if args.rows == "all" else \
        set() if args.rows == "none" else set(args.rows.split(","))
    n = int(args.n)
    nsteps = 50

    log(f"[bench] headline: {n} particles, {nsteps} RK2 steps per pass, SoA")
    ps = soax.ParticleSet(si.BASE_FIELDS, n)
    ps.fill(seed=0, vel_mode=1, abc=[1, 1, 1])
    ps.soa_to_aos()
    for _ in range(args.warmup):
        ps.step("soa", "rk2_abc", 1e-3, nsteps, abc=[1, 1, 1], wrap=True)
    torch.cuda.synchronize()
    with Timer(torch) as t:
        for _ in range(args.steps):
            ps.step("soa", "rk2_abc", 1e-3, nsteps, abc=[1, 1, 1], wrap=True)
    value = rate(n * nsteps * args.steps, t.ms)
    ms_per_step = t.ms / args.steps
    per_launch = t.ms / (args.steps * nsteps)
    log(f"[bench] SoA RK2: {value:.4e} updates/s, {per_launch:.3f} ms/launch")

    kname = "soa_step_kernel<RK2_ABC,double,float,2>"
    traffic = traffic_from_profiles(kname, "hbm_bytes_per_launch")
    roofline = {"kernel": kname, "bound": "hbm", "achieved": gbs(60 * n, per_launch),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs(60 * n, per_launch) / HBM_PEAK_GBS,
                "traffic": traffic, "alg_bytes_per_launch": 60 * n,
                "ms_per_launch": per_launch}

    out_rows = {}
    if "aos" in rows:
        log("[bench] RK2 AoS (LDS-staged) and naive AoS")
        out_rows["rk2_aos"] = bench_rk2(torch, soax, ps, n, nsteps, "aos", 1)
        out_rows["rk2_aos_naive"] = bench_rk2(torch, soax, ps, n, nsteps, "aos_naive", 1)
        out_rows["rk2_soa_over_aos"] = value / out_rows["rk2_aos"]["updates_per_s"]
        out_rows["rk2_soa_over_aos_naive"] = value / out_rows["rk2_aos_naive"]["updates_per_s"]
    if "euler" in rows:
        log("[bench] Euler at the headline size, every layout")
        for lay in ("soa", "aos", "aos_naive"):
            out_rows[f"euler_{lay}"] = bench_euler(torch, soax, ps, n, 20, lay)
        out_rows["euler_soa_over_aos"] = (out_rows["euler_soa"]["updates_per_s"] /
                                          out_rows["euler_aos"]["updates_per_s"])
    if "integrators" in rows:
        log("[bench] Heun and RK4 steps at the headline size")
        out_rows["integrators"] = bench_integrators(torch, soax, ps, n)
    if "fused" in rows:
        log("[bench] extra: all steps of a job in one launch (particles held in registers)")
        out_rows["fused_extra"] = bench_fused(torch, soax, si, ps, n, nsteps, ms_per_step)
    ps.close()
    del ps
    torch.cuda.empty_cache()
    if "aosoa" in rows:
        log("[bench] tiled (AoSoA) copy of the headline set")
        out_rows["aosoa"] = bench_aosoa(torch, soax, si, n)
    if "small" in rows:
        log("[bench] 1e5-particle Euler workload")
        out_rows["euler_1e5"] = bench_small_euler(torch, soax, si)
    if "copy" in rows:
        log("[bench] copy ceiling")
        out_rows["copy"] = bench_copy(torch, soax)
    if "probes" in rows:
        log("[bench] stream probes: the step patterns without arithmetic")
        out_rows["probes"] = bench_probes(torch, soax, n)
        probe = out_rows["probes"]["rk2"]["GBps"]
        roofline["pattern_ceiling"] = {"probe": "soax_probe rk2 (same loads and stores, no "
                                                "arithmetic)", "GBps": probe,
                                       "frac_of_probe": roofline["achieved"] / probe}
        if "euler_soa" in out_rows:
            out_rows["euler_soa"]["frac_of_probe"] = (out_rows["euler_soa"]["physical_GBps"] /
                                                      out_rows["probes"]["euler"]["GBps"])
    if "wide" in rows:
        log("[bench] wide record: transposes and Euler with acceleration")
        out_rows["wide"] = bench_wide(torch, soax, si, 30_000_000)
    if "adjoint" in rows:
        log("[bench] RK2 forward and forward + adjoint")
        out_rows["adjoint"] = bench_adjoint(torch, soax, si, 10_000_000)
    if "batch" in rows:
        log("[bench] batched sets")
        out_rows["batch"] = bench_batch(torch, soax, si)
    if "remove" in rows:
        log("[bench] removal by overwriting with the last particle")
        out_rows["remove"] = bench_remove(torch, soax, si, n)
    if "expr" in rows:
        log("[bench] fused array expressions")
        out_rows["expr"] = bench_expr(torch, soax, si, n)
    if "expr_euler" in rows:
        log("[bench] generated Euler update vs the hand-written step")
        out_rows["expr_euler"] = bench_expr_euler(torch, soax, si)
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        import oracle as ref
        log("[bench] oracle CPU baseline")
        cpu = cpu_baseline(ref, si)

    line = {"metric": METRIC, "value": value, "unit": "particle-updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic (seeded SplitMix64 fill on the GPU)",
            "config": {"workload": f"{n:.0e} particles {{int32 id; fp64 pos[3]; fp32 vel[3]}}, "
                                   f"{nsteps} RK2 steps per pass in the ABC field A=B=C=1, "
                                   "dt=1e-3, periodic wrap, SoA layout",
                       "n": n, "nsteps_per_pass": nsteps, "layout": "soa",
                       "parallelism": "none (1 GPU)"},
            "roofline": roofline, "cpu_baseline": cpu, "rows": out_rows,
            "device": torch.cuda.get_device_name(0)}
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
