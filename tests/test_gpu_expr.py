"""GPU parity of the fused array expressions against the oracle's
element-by-element evaluation (Section 4.1's whole-array expressions):
bit-exact for every op (each is one correctly rounded double operation on
both sides), on set arrays and plain tensors, at ragged sizes, in place,
and at sizes that take the streaming kernel."""
import numpy as np
import pytest
import torch

import oracle as ref
import synth_inputs as si

pytestmark = pytest.mark.gpu

soax = pytest.importorskip("paper_1710_03462_amd")
from paper_1710_03462_amd import expr as E  # noqa: E402


def bits_equal(a, b):
    """Same type, NaN in the same places (their payloads may differ between
    the CPU and the GPU), every other element bit for bit."""
    if a.dtype != b.dtype or a.shape != b.shape:
        return False
    na, nb = np.isnan(a), np.isnan(b)
    if not np.array_equal(na, nb):
        return False
    return np.array_equal(a[~na].view(np.uint8), b[~nb].view(np.uint8))


@pytest.mark.parametrize("n", [1, 255, 256, 257, 100_003])
def test_paper_example_on_a_set(n):
    fields = si.BASE_FIELDS
    arrays = si.random_state(fields, n, n)
    ps = soax.ParticleSet(fields, n)
    ps.upload_soa(arrays)
    sch = ps.schema
    ps.assign(("pos", 0), ps.arr("vel", 1) - ps.arr("vel", 2))
    torch.cuda.synchronize()
    v1, v2 = sch.array_index("vel", 1), sch.array_index("vel", 2)
    want = ref.eval_program(arrays, [(ref.OP_ARRAY, v1, 0), (ref.OP_ARRAY, v2, 0),
                                     (ref.OP_SUB, 0, 0)])
    got = ps.download_soa()
    assert bits_equal(got[sch.array_index("pos", 0)], want)
    for a in range(len(arrays)):  # nothing else changed
        if a != sch.array_index("pos", 0):
            assert bits_equal(got[a], arrays[a])
    ps.close()


PROGRAMS = {
    # x = sqrt(|a*b + 1.5/c|) - min(d, max(e, -f)) + (2 - a)
    "all_ops": lambda a, b, c, d, e, f: (E.sqrt(abs(a * b + 1.5 / c)) - E.minimum(d, E.maximum(e, -f))
                                         + (2.0 - a)),
    "kinetic": lambda a, b, c, d, e, f: 0.5 * f * (a * a + b * b + c * c),
    "ratio": lambda a, b, c, d, e, f: (a - b) / (c * c + 3.0) * d - e,
}
TYPES = [np.int8, np.uint8, np.int32, np.int64, np.float32, np.float64]


def make_sources(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for t in TYPES:
        if np.issubdtype(t, np.integer):
            info = np.iinfo(t)
            out.append(rng.integers(max(info.min, -1000), min(info.max, 1000), n, dtype=t,
                                    endpoint=True))
        else:
            out.append((rng.standard_normal(n) * 3).astype(t))
    return out


def to_ops(ex, keys):
    return ex.as_tuples(lambda k: next(j for j, kk in enumerate(keys) if kk is k))


@pytest.mark.parametrize("name", list(PROGRAMS))
@pytest.mark.parametrize("dst_t", [np.float32, np.float64])
@pytest.mark.parametrize("n", [7, 4099, 65_536])
def test_programs_on_tensors(name, dst_t, n):
    host = make_sources(n, n)
    dev = [torch.from_numpy(h).cuda() for h in host]
    leaves = [E.array(t) for t in dev]
    ex = PROGRAMS[name](*leaves)
    dst = torch.empty(n, dtype=torch.float32 if dst_t == np.float32 else torch.float64, device="cuda")
    soax.evaluate(dst, ex)
    torch.cuda.synchronize()
    keys = ex.keys()
    want = ref.eval_program([host[next(j for j, t in enumerate(dev) if t is k)] for k in keys],
                            to_ops(ex, keys), dst_t)
    assert bits_equal(dst.cpu().numpy(), want)


@pytest.mark.parametrize("name", list(PROGRAMS))
@pytest.mark.parametrize("dst_t", [np.float32, np.float64])
def test_programs_on_tensors_streaming_size(name, dst_t):
    # every source type at a footprint above 128 MB (5e6 x 30-34 bytes): the
    # kernel that moves each element through buffer windows
    n = 5_000_003
    host = make_sources(n, 11)
    dev = [torch.from_numpy(h).cuda() for h in host]
    leaves = [E.array(t) for t in dev]
    ex = PROGRAMS[name](*leaves)
    dst = torch.empty(n, dtype=torch.float32 if dst_t == np.float32 else torch.float64, device="cuda")
    soax.evaluate(dst, ex)
    torch.cuda.synchronize()
    keys = ex.keys()
    want = ref.eval_program([host[next(j for j, t in enumerate(dev) if t is k)] for k in keys],
                            to_ops(ex, keys), dst_t)
    assert bits_equal(dst.cpu().numpy(), want)


def test_in_place_update_and_repeat():
    n = 10_007
    x = torch.linspace(-3, 3, n, dtype=torch.float64, device="cuda")
    v = torch.linspace(1, 2, n, dtype=torch.float32, device="cuda")
    hx, hv = x.cpu().numpy(), v.cpu().numpy()
    ex = E.array(x) + 1e-3 * E.array(v)  # x += dt v, one kernel
    for _ in range(3):
        soax.evaluate(x, ex)
        hx = ref.eval_program([hx, hv], [(ref.OP_ARRAY, 0, 0), (ref.OP_CONST, 0, 1e-3),
                                         (ref.OP_ARRAY, 1, 0), (ref.OP_MUL, 0, 0),
                                         (ref.OP_ADD, 0, 0)])
    torch.cuda.synchronize()
    assert bits_equal(x.cpu().numpy(), hx)


def test_streaming_size_sampled():
    # 1.2e7 doubles x 3 arrays > 128 MB: the streaming kernel
    n = 12_000_001
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    a = torch.randn(n, generator=g, dtype=torch.float64, device="cuda")
    b = torch.rand(n, generator=g, dtype=torch.float64, device="cuda") + 0.5
    out = torch.empty_like(a)
    A, B = E.array(a), E.array(b)
    soax.evaluate(out, E.sqrt(A * A + B) / B)
    torch.cuda.synchronize()
    idx = np.concatenate([np.arange(0, 1000), np.arange(n - 1000, n),
                          np.random.default_rng(0).integers(0, n, 5000)])
    ti = torch.from_numpy(idx).cuda()
    ha, hb = a[ti].cpu().numpy(), b[ti].cpu().numpy()
    want = ref.eval_program([ha, hb], [(0, 0, 0), (0, 0, 0), (ref.OP_MUL, 0, 0), (0, 1, 0),
                                       (ref.OP_ADD, 0, 0), (ref.OP_SQRT, 0, 0), (0, 1, 0),
                                       (ref.OP_DIV, 0, 0)])
    assert bits_equal(out[ti].cpu().numpy(), want)


def test_empty_and_errors():
    z = torch.empty(0, dtype=torch.float64, device="cuda")
    soax.evaluate(z, E.array(z) * 2.0)  # n = 0: compiles, launches nothing
    i = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        soax.evaluate(i, E.array(i) + 1.0)
    ps = soax.ParticleSet(si.BASE_FIELDS, 10)
    with pytest.raises(soax.SoaxError):
        ps.assign(("id", 0), ps.arr("vel", 0) * 2.0)  # integer destination
    ps.close()


@pytest.mark.parametrize("n", [257, 100_003, 4_000_003])
def test_generated_euler_update_equals_the_step_kernel(n):
    """The Euler update written as three generated expressions,
    pos_d = pos_d + dt * vel_d (Section 4.2.2 compares this form with the
    hand-written SoA loop), gives the step kernel's results bit for bit: both
    are one double multiply and one double add per component; the oracle's
    Euler step without wrap agrees too."""
    fields, dt, steps = si.BASE_FIELDS, 1e-3, 7
    arrays = si.random_state(fields, n, seed=n + 3)
    gen = soax.ParticleSet(fields, n, aos=False)
    hand = soax.ParticleSet(fields, n, aos=False)
    gen.upload_soa(arrays)
    hand.upload_soa(arrays)
    progs = [gen.arr("pos", d) + dt * gen.arr("vel", d) for d in range(3)]
    for _ in range(steps):
        for d in range(3):
            gen.assign(("pos", d), progs[d])
    hand.step("soa", "euler", dt, steps, wrap=False)
    torch.cuda.synchronize()
    got, want_gpu = gen.download_soa(), hand.download_soa()
    want = [a.copy() for a in arrays]
    ref.step_soa(ref.Schema(fields), want, ref.EULER, dt, steps, wrap=False)
    for a in range(len(arrays)):
        assert np.array_equal(got[a], want_gpu[a]), a
        assert np.array_equal(got[a], want[a]), a
    gen.close()
    hand.close()
