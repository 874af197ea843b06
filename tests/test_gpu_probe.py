"""The bandwidth probes (soax_probe) move exactly the bytes they claim: the
RK2 pattern rewrites the positions unchanged and stores them, rounded to
float, as velocities; the Euler pattern rewrites the positions unchanged;
the read pattern changes nothing; the write pattern stores zeros.  A ragged
size checks the tail of the grid."""
import pytest
import torch

pytestmark = pytest.mark.gpu

soax = pytest.importorskip("paper_1710_03462_amd")


def arrays(n, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    pos = [torch.rand(n, dtype=torch.float64, device="cuda", generator=g) * 6.0 for _ in range(3)]
    vel = [torch.randn(n, dtype=torch.float32, device="cuda", generator=g) for _ in range(3)]
    return pos, vel


@pytest.mark.parametrize("n", [1, 129, 100_003])
def test_probe_patterns(n):
    pos, vel = arrays(n, n)
    p0, v0 = [t.clone() for t in pos], [t.clone() for t in vel]
    soax.probe("read", pos)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(pos + vel, p0 + v0))
    soax.probe("euler", pos, vel)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(pos + vel, p0 + v0))
    soax.probe("rk2", pos, vel)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(pos, p0))
    assert all(torch.equal(v, p.to(torch.float32)) for v, p in zip(vel, p0))
    soax.probe("write", pos, vel)
    torch.cuda.synchronize()
    assert all(int(torch.count_nonzero(t)) == 0 for t in pos + vel)
