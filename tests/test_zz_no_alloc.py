"""qw_step_noalloc, the stepping entry point that allocates nothing: its
ping-pong buffer is the library's fixed per-device array instead of the
plan's scratch. Checked through the C ABI against qw_step (same kernels, so
bit for bit), on two calls in a row with the second on a smaller field, from
a fresh process or after any other test; size limits and argument errors are
refused on the host."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

LIMIT = 64 << 20


@pytest.fixture(scope="module")
def qw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1603_06442_amd import qw as mod
    return mod


def field(plan, seed):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(plan.shape) + 1j * rng.standard_normal(plan.shape)
    return torch.from_numpy(z / np.linalg.norm(z)).to(plan.torch_dtype).cuda()


@pytest.mark.parametrize("first,second", [
    # 3D complex64 at the limit (128^3: exactly 64 MiB, the plane-ring kernel),
    # then a smaller 3D complex128 field (one thread per site)
    ((3, (128, 128, 128), "c64", 0.05, 5), (3, (16, 32, 64), "c128", 0.3, 3)),
    # 2D complex64, then a smaller 2D field in complex128
    ((2, (512, 256), "c64", 0.2, 4), (2, (64, 32), "c128", 0.0, 7)),
    # 1D four-step length (streams through the buffer), then one that stays on chip
    ((1, (65536,), "c128", 0.1, 3), (1, (4096,), "c128", 0.1, 6)),
])
def test_noalloc_step_equals_qw_step(qw, first, second):
    for k, (d, shape, dtype, m, nsteps) in enumerate((first, second)):
        plan = qw.Plan(d, list(shape), m, dtype)
        x0 = field(plan, 10 + k)
        a = x0.clone()
        plan.step(a, nsteps)
        b = x0.clone()
        plan.step_noalloc(b, nsteps)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (d, shape, dtype, nsteps)
        # the buffer keeps the last call's contents; a second call on the
        # result continues the evolution exactly as qw_step does
        plan.step(a, 2)
        plan.step_noalloc(b, 2)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (d, shape, dtype)


def test_noalloc_step_under_graph_capture(qw):
    """A plan whose first stepping call is captured: the captured
    qw_step_noalloc needs no allocation, and every replay (with eager work
    and synchronisation between replays) gives the eager qw_step result."""
    shape = (32, 32, 64)
    plan = qw.Plan(3, list(shape), 0.1, "c64")
    x0 = field(plan, 3)
    ga = x0.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.step_noalloc(ga, 3, stream=torch.cuda.current_stream())
    ref = qw.Plan(3, list(shape), 0.1, "c64")
    want = x0.clone()
    ref.step(want, 3)
    for r in range(3):
        ga.copy_(x0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ga, want), r
        e = x0.clone()
        ref.step(e, 1)
        torch.cuda.synchronize()


def test_noalloc_step_refuses_fields_beyond_the_buffer(qw):
    # 3D complex128 128^3 is 128 MiB: twice the buffer
    plan = qw.Plan(3, [128, 128, 128], 0.1, "c128")
    assert 4 * 128 ** 3 * 16 > LIMIT
    x = plan.empty()
    with pytest.raises(qw.QwError) as e:
        plan.step_noalloc(x, 1)
    assert e.value.status == qw.QW_ERR_UNSUPPORTED
    small = qw.Plan(3, [8, 8, 8], 0.1, "c64")
    with pytest.raises(qw.QwError) as e:
        small.step_noalloc(small.empty(), -1)
    assert e.value.status == qw.QW_ERR_INVALID
