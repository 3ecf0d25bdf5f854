"""GPU parity of the 7 x 7 filter stencil (sec. 6, "filter size 7").

Every output is the float32 fused multiply-add chain of the definition, so
the comparison with the oracle is bit-exact: the wavefront-strip tile
kernel for every tile height / wavefront count (including strips of unequal
length), tiles ragged on all four sides, the generic and dynamic kernels,
and the paper's size grid N = 64 .. 2048 (full grids up to 512, sampled row
bands above, where the oracle runs on the band and its three-row halo).
"""
import sys

import numpy as np
import pytest

import synth
from oracle import bodies
from paper_2209_10643_amd import helpers as H
from paper_2209_10643_amd import upir as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def note(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    U.lib()
    s = torch.cuda.Stream()
    prev = torch.cuda.current_stream()
    torch.cuda.set_stream(s)  # torch's work and the library's are ordered on one stream
    c = H.Context(0, stream=s)
    yield c
    c.close()
    torch.cuda.set_stream(prev)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def weights(seed):
    return synth.uniform_pm1(seed, 99, 49).reshape(7, 7) * np.float32(0.25)


def run_filter(ctx, src, w, sched=None, spmd=None, box=None):
    Hh, W = src.shape
    ts, tw = dev(src), dev(w)
    td = torch.full((Hh, W), -7.0, device="cuda")
    args = U.upir_filter7_args(ts.data_ptr(), td.data_ptr(), tw.data_ptr(), W)
    dims = box or [(3, Hh - 3, 1), (3, W - 3, 1)]
    lp = ctx.loop(U.UPIR_BODY_FILTER7, args, dims, sched)
    variant = U.VARIANTS[ctx.resolve(lp, spmd)[2]]
    ctx.launch(lp, spmd)
    ctx.sync()
    out = td.cpu().numpy()
    ctx.free(lp)
    return out, variant


CASES = [
    ((64, 64), None, None, "filter7_tile"),
    ((300, 520), None, None, "filter7_tile"),
    ((203, 780), H.make_sched(U.UPIR_SCHED_STATIC, tile=(4, 256)), H.make_spmd(0, 64), "filter7_tile"),
    ((203, 780), H.make_sched(U.UPIR_SCHED_STATIC, tile=(16, 256)), H.make_spmd(0, 192), "filter7_tile"),
    ((203, 780), H.make_sched(U.UPIR_SCHED_STATIC, tile=(64, 256)), H.make_spmd(0, 512), "filter7_tile"),
    ((203, 780), H.make_sched(U.UPIR_SCHED_STATIC, tile=(32, 256)), H.make_spmd(5, 128), "filter7_tile"),
    ((203, 780), H.make_sched(U.UPIR_SCHED_STATIC_CHUNK, 3, tile=(8, 256)), H.make_spmd(4, 256), "filter7_tile"),
    ((7, 8), None, None, "filter7_tile"),                                      # one output row of two points
    ((7, 1028), None, None, "filter7_tile"),                                   # one output row
    ((500, 8), None, None, "filter7_tile"),                                    # two output columns
    ((70, 77), None, None, "generic"),                                         # pitch % 4 != 0
    ((90, 100), H.make_sched(U.UPIR_SCHED_STATIC), H.make_spmd(9, 64), "generic"),
    ((90, 100), H.make_sched(U.UPIR_SCHED_DYNAMIC, 2), H.make_spmd(7, 64), "dynamic"),
]


@pytest.mark.parametrize("shape,sched,spmd,variant", CASES)
def test_filter7_parity(ctx, shape, sched, spmd, variant):
    note(f"filter7 {shape} {variant}")
    src = synth.uniform_pm1(40, 0, shape[0] * shape[1]).reshape(shape)
    w = weights(40)
    got, v = run_filter(ctx, src, w, sched, spmd)
    assert v == variant
    want = bodies.filter7(src, w, np.full(shape, -7.0, np.float32))
    assert np.array_equal(got, want)


def test_filter7_sub_box(ctx):
    """A loop box inside the interior: only the box is written."""
    src = synth.uniform_pm1(41, 0, 120 * 600).reshape(120, 600)
    w = weights(41)
    box = [(10, 97, 1), (260, 517, 1)]
    got, v = run_filter(ctx, src, w, H.make_sched(U.UPIR_SCHED_STATIC, tile=(16, 256)), None, box)
    assert v == "filter7_tile"
    full = bodies.filter7(src, w, np.full(src.shape, -7.0, np.float32))
    want = np.full(src.shape, -7.0, np.float32)
    want[10:97, 260:517] = full[10:97, 260:517]
    assert np.array_equal(got, want)


@pytest.mark.parametrize("N", [64, 128, 256, 512, 1024, 2048])
def test_filter7_paper_grid(ctx, N):
    note(f"filter7 paper grid N={N}")
    src = synth.uniform_01(42, N, N * N).reshape(N, N)
    w = weights(42)
    got, v = run_filter(ctx, src, w)
    assert v == "filter7_tile"
    if N <= 512:
        assert np.array_equal(got, bodies.filter7(src, w, np.full((N, N), -7.0, np.float32)))
    else:
        for a in list(range(3, N - 3, N // 7)) + [N - 19]:   # bands of 16 rows, the last one at the edge
            b = min(a + 16, N - 3)
            band = bodies.filter7(src[a - 3:b + 3], w)       # rows a .. b-1 exact
            assert np.array_equal(got[a:b, 3:N - 3], band[3:-3, 3:-3]), a
        assert (got[:3] == -7.0).all() and (got[N - 3:] == -7.0).all()
