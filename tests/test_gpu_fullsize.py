"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times.

The GPU fills its own state (seeded fill); the oracle fills sampled ranges of
particles independently (every fill value depends on the particle index only)
and advances them.  Sampled particles are compared with the oracle; whole
arrays are checked on the GPU through properties that hold at any size: the
SoA and AoS paths agree bit for bit, untouched fields are unchanged, round
trips are the identity, the graph and per-set launches agree, gradients are
additive over particles and independent of the checkpoint interval."""
import numpy as np
import pytest
import torch

import synth_inputs as si
from gpu_util import assert_fields_close, assert_positions_close, ulp_distance

pytestmark = pytest.mark.gpu

soax = pytest.importorskip("paper_1710_03462_amd")


def sample_ranges(n, width=128, extra=4, seed=0):
    rng = np.random.default_rng(seed)
    starts = [0, max(0, n // 2 - width // 2), max(0, n - width)]
    starts += [int(s) for s in rng.integers(0, max(1, n - width), extra)]
    return [(s, min(width, n - s)) for s in sorted(set(starts))]


def gpu_slice(ps, r0, cnt):
    return [t[r0:r0 + cnt].cpu().numpy() for t in ps.soa]


def test_rk2_headline_1e8(ref):
    n, nsteps, abc = 100_000_000, 50, [1.0, 1.0, 1.0]
    fields = si.BASE_FIELDS
    sch = ref.Schema(fields)
    ps = soax.ParticleSet(fields, n)
    ps.fill(seed=0, vel_mode=1, abc=abc)
    ps.soa_to_aos()
    ranges = sample_ranges(n)
    init = {}
    for r0, cnt in ranges:
        want = ref.fill_range(sch, r0, cnt, seed=0, vel_mode=1, abc=abc)
        got = gpu_slice(ps, r0, cnt)
        for a in range(4):
            assert np.array_equal(got[a], want[a]), (r0, a)
        for a in range(4, 7):
            assert ulp_distance(got[a], want[a]).max() <= 1
        init[r0] = want
    ps.step("soa", "rk2_abc", 1e-3, nsteps, abc=abc, wrap=True)
    ps.step("aos", "rk2_abc", 1e-3, nsteps, abc=abc, wrap=True)
    torch.cuda.synchronize()
    # the SoA and AoS paths run the same arithmetic: bit-identical everywhere
    rec = ps.aos[: n * ps.stride].view(n, ps.stride)
    for d in range(3):
        pos_aos = rec[:, 8 + 8 * d: 16 + 8 * d].contiguous().view(torch.float64).view(-1)
        vel_aos = rec[:, 32 + 4 * d: 36 + 4 * d].contiguous().view(torch.float32).view(-1)
        assert torch.equal(pos_aos, ps.soa[1 + d])
        assert torch.equal(vel_aos, ps.soa[4 + d])
    ids = rec[:, 0:4].contiguous().view(torch.int32).view(-1)
    assert torch.equal(ids, ps.soa[0])
    assert torch.equal(ps.soa[0], torch.arange(n, dtype=torch.int32, device="cuda"))
    for d in range(3):
        assert float(ps.soa[1 + d].min()) >= 0.0 and float(ps.soa[1 + d].max()) < si.BOX_L
    for r0, cnt in ranges:
        want = [a.copy() for a in init[r0]]
        ref.step_soa(sch, want, ref.RK2_ABC, 1e-3, nsteps, abc=abc, wrap=True)
        got = gpu_slice(ps, r0, cnt)
        for d in range(3):
            assert_positions_close(got[1 + d], want[1 + d])
            assert_fields_close(got[4 + d], want[4 + d])
    ps.close()


def test_integrator_variants_1e8(ref):
    """Heun and RK4 on the headline set, as the benchmark's integrator row
    runs them (SoA, then the LDS-staged AoS copy), sampled against the oracle."""
    n, abc = 100_000_000, [1.0, 1.0, 1.0]
    fields = si.BASE_FIELDS
    sch = ref.Schema(fields)
    ps = soax.ParticleSet(fields, n)
    ps.fill(seed=0, vel_mode=1, abc=abc)
    ps.soa_to_aos()
    ranges = sample_ranges(n, width=64)
    init = {r0: ref.fill_range(sch, r0, cnt, seed=0, vel_mode=1, abc=abc) for r0, cnt in ranges}
    ps.step("soa", "heun_abc", 1e-3, 3, abc=abc, wrap=True)
    ps.step("soa", "rk4_abc", 1e-3, 3, abc=abc, wrap=True)
    ps.step("aos", "heun_abc", 1e-3, 3, abc=abc, wrap=True)
    ps.step("aos", "rk4_abc", 1e-3, 3, abc=abc, wrap=True)
    torch.cuda.synchronize()
    rec = ps.aos[: n * ps.stride].view(n, ps.stride)
    for d in range(3):  # the two layouts ran the same arithmetic
        pos_aos = rec[:, 8 + 8 * d: 16 + 8 * d].contiguous().view(torch.float64).view(-1)
        assert torch.equal(pos_aos, ps.soa[1 + d])
    del rec, pos_aos
    for r0, cnt in ranges:
        want = [a.copy() for a in init[r0]]
        ref.step_soa(sch, want, ref.HEUN_ABC, 1e-3, 3, abc=abc, wrap=True)
        ref.step_soa(sch, want, ref.RK4_ABC, 1e-3, 3, abc=abc, wrap=True)
        got = gpu_slice(ps, r0, cnt)
        for d in range(3):
            assert_positions_close(got[1 + d], want[1 + d])
            assert_fields_close(got[4 + d], want[4 + d])
    ps.close()


def test_tiled_copy_1e8():
    """The benchmark's AoSoA rows at the headline size: Euler and RK2 steps on
    the tiled copy give the SoA kernels' results bit for bit (whole arrays)."""
    n, abc = 100_000_000, [1.0, 1.0, 1.0]
    ps = soax.ParticleSet(si.BASE_FIELDS, n, aos=False, aosoa=True)
    ps.fill(seed=0, vel_mode=1, abc=abc)
    ps.soa_to_aosoa()
    for integ, steps in (("euler", 2), ("rk2_abc", 3)):
        ps.step("aosoa", integ, 1e-3, steps, abc=abc, wrap=True)
        ps.step("soa", integ, 1e-3, steps, abc=abc, wrap=True)
    stepped = [t.clone() for t in ps.soa[1:]]
    ps.aosoa_to_soa()
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(ps.soa[1:], stepped))
    assert torch.equal(ps.soa[0], torch.arange(n, dtype=torch.int32, device="cuda"))
    del stepped
    ps.close()


def test_wide_record_transposes_and_steps_3e7(ref):
    n = 30_000_000
    fields = si.WIDE_FIELDS
    sch = ref.Schema(fields)
    ps = soax.ParticleSet(fields, n)
    ps.fill(seed=0)
    ranges = sample_ranges(n)
    gpu_init = {r0: gpu_slice(ps, r0, cnt) for r0, cnt in ranges}
    ref_init = {r0: ref.fill_range(sch, r0, cnt, seed=0) for r0, cnt in ranges}
    normals = set(range(sch.array_index("vel"), sch.array_index("acc") + 3))
    for r0, _ in ranges:
        for a, (g, w) in enumerate(zip(gpu_init[r0], ref_init[r0])):
            if a in normals:
                assert ulp_distance(g, w).max() <= 1
            else:
                assert np.array_equal(g, w)
    ps.soa_to_aos()
    aos0 = ps.aos[: n * ps.stride].clone()
    filled = [t.clone() for t in ps.soa]
    for t in ps.soa:
        t.zero_()
    ps.aos_to_soa()
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(ps.soa, filled))
    ps.soa_to_aos()
    torch.cuda.synchronize()
    assert torch.equal(ps.aos[: n * ps.stride], aos0)  # AoS -> SoA -> AoS is the identity
    del filled
    ps.step("soa", "euler_acc", 1e-3, 20, wrap=True)
    ps.soa_to_aos()
    torch.cuda.synchronize()
    rec = ps.aos[: n * ps.stride].view(n, ps.stride)
    rec0 = aos0.view(n, ps.stride)
    offs, _, _ = ps.schema.layout()
    untouched = [(offs[0], 8), (offs[1], 4), (offs[4], 12), (offs[5], 9)]  # tag, id, acc, mass+flags
    for off, nb in untouched:
        assert torch.equal(rec[:, off:off + nb], rec0[:, off:off + nb])
    del aos0, rec0
    pos = range(sch.array_index("pos"), sch.array_index("pos") + 3)
    for r0, cnt in ranges:
        want = [a.copy() for a in ref_init[r0]]
        ref.step_soa(sch, want, ref.EULER_ACC, 1e-3, 20, wrap=True)
        got = gpu_slice(ps, r0, cnt)
        # Box-Muller values may differ by an ulp between libm and the device:
        # particles whose whole initial state agrees must match bit for bit
        same = np.ones(cnt, bool)
        for g, w in zip(gpu_init[r0], ref_init[r0]):
            same &= g == w
        assert same.mean() > 0.9
        for a in range(len(want)):
            assert np.array_equal(got[a][same], want[a][same]), a
            if same.all():
                continue
            if a in pos:
                assert_positions_close(got[a][~same], want[a][~same], tol=1e-7)
            elif a in normals:
                assert_fields_close(got[a][~same], want[a][~same])


def test_adjoint_1e7_200_steps(ref):
    n, nsteps, dt, k = 10_000_000, 200, 5e-3, 20
    abc = [1.0, 0.8, 0.6]
    x0, target = si.adjoint_inputs(n, seed=0)
    abc_host = soax.autograd._host3(torch.tensor(abc, dtype=torch.float64))
    X0 = torch.from_numpy(x0).cuda()
    TG = torch.from_numpy(target).cuda()
    xT, tape = soax.forward_ckpt(X0, abc_host, dt, nsteps, k)
    loss, lam = soax.sqdist_loss(xT, TG)
    gx, gabc = soax.adjoint(tape, lam, abc_host, dt, nsteps, k)
    torch.cuda.synchronize()
    # sampled particles against the oracle, which stores every state
    for r0, cnt in sample_ranges(n, width=64):
        sl = slice(r0, r0 + cnt)
        rxT = ref.rk2_forward(x0[:, sl], abc, dt, nsteps)
        _, rlam = ref.sqdist_loss(rxT, target[:, sl])
        rgx, _ = ref.adjoint(x0[:, sl], rlam, abc, dt, nsteps)
        assert np.abs(xT[:, sl].cpu().numpy() - rxT).max() <= 1e-12 * si.BOX_L
        g = gx[:, sl].cpu().numpy()
        assert np.abs(g - rgx).max() <= 1e-6 * np.abs(rgx).max()
    # the parameter gradient is a sum over particles: two halves add up
    h = n // 2
    parts = []
    for sl in (slice(0, h), slice(h, n)):
        xa, ta = soax.forward_ckpt(X0[:, sl].contiguous(), abc_host, dt, nsteps, k)
        _, la = soax.sqdist_loss(xa, TG[:, sl].contiguous())
        parts.append(soax.adjoint(ta, la, abc_host, dt, nsteps, k)[1])
    total = (parts[0] + parts[1]).cpu().numpy()
    g = gabc.cpu().numpy()
    assert np.all(np.abs(total - g) <= 1e-10 * np.abs(g))
    # ... and does not depend on the checkpoint interval
    xT2, tape2 = soax.forward_ckpt(X0, abc_host, dt, nsteps, 10)
    gx2, gabc2 = soax.adjoint(tape2, lam, abc_host, dt, nsteps, 10)
    assert torch.equal(gx2, gx) and torch.equal(gabc2, gabc) and torch.equal(xT2, xT)


def test_batch_256_uneven_sets(ref):
    sizes, dts, abc = si.batch_plan(256, seed=0)
    sets = []
    for s, n in enumerate(sizes):
        ps = soax.ParticleSet(si.BASE_FIELDS, int(n), aos=False)
        ps.fill(seed=s, vel_mode=1, abc=abc[s])
        sets.append(ps)
    start = [[t.clone() for t in ps.soa[1:]] for ps in sets]
    b = soax.Batch(sets)
    b.tune()
    b.step(dts, abc, 100, mode=soax.GRAPH)
    torch.cuda.synchronize()
    graph = [[t.clone() for t in ps.soa[1:]] for ps in sets]
    for ps, st in zip(sets, start):
        for t, s0 in zip(ps.soa[1:], st):
            t.copy_(s0)
    b.step(dts, abc, 100, mode=soax.PER_SET)
    torch.cuda.synchronize()
    for ps, g in zip(sets, graph):
        assert all(torch.equal(t, x) for t, x in zip(ps.soa[1:], g))
    sch = ref.Schema(si.BASE_FIELDS)
    order = np.argsort(sizes)
    picks = sorted(set([int(order[0]), int(order[-1])] +
                       [int(x) for x in np.random.default_rng(1).integers(0, 256, 6)]))
    for s in picks:
        n = int(sizes[s])
        for r0, cnt in sample_ranges(n, width=64, extra=1, seed=s):
            init = ref.fill_range(sch, r0, cnt, seed=s, vel_mode=1, abc=abc[s])
            want = [a.copy() for a in init]
            ref.step_soa(sch, want, ref.RK2_ABC, dts[s], 100, abc=abc[s], wrap=True)
            got = [t[r0:r0 + cnt].cpu().numpy() for t in sets[s].soa]
            for d in range(3):
                assert_positions_close(got[1 + d], want[1 + d])
                assert_fields_close(got[4 + d], want[4 + d])
    b.close()


def test_maximum_particle_count_soa(ref):
    """n = 2^31 - 1, the library's limit (86 GB of SoA arrays): the fill, an
    Euler step and an RK2 step index past 2^31 elements and 2^34 bytes; the
    first and last particles are compared with the oracle."""
    n = 2 ** 31 - 1
    fields = si.BASE_FIELDS
    sch = ref.Schema(fields)
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 100 * 2 ** 30:
        pytest.skip("needs about 90 GB of free device memory")
    ps = soax.ParticleSet(fields, n, aos=False)
    ps.fill(seed=3)
    ps.step("soa", "euler", 1e-3, 1, wrap=True)
    ps.step("soa", "rk2_abc", 1e-3, 1, abc=[1.0, 1.0, 1.0], wrap=True)
    torch.cuda.synchronize()
    for r0, cnt in [(0, 64), (2 ** 31 - 4096, 4096 - 1), (n - 64, 64)]:
        want = ref.fill_range(sch, r0, cnt, seed=3)
        got0 = gpu_slice(ps, r0, cnt)
        assert np.array_equal(got0[0], np.arange(r0, r0 + cnt, dtype=np.int32))
        ref.step_soa(sch, want, ref.EULER, 1e-3, 1, wrap=True)
        ref.step_soa(sch, want, ref.RK2_ABC, 1e-3, 1, abc=[1.0, 1.0, 1.0], wrap=True)
        for d in range(3):
            assert_positions_close(got0[1 + d], want[1 + d])
            assert_fields_close(got0[4 + d], want[4 + d])
    ps.close()
    del ps
    torch.cuda.empty_cache()
