"""GPU parity of the MFMA matmul loop (float32, bfloat16, split bfloat16).

Integer matrices with entries in {-2..2} are exact in every variant, so
they pin the MFMA fragment layouts bit for bit. Random normal matrices are
checked normwise against the float64 product: float32 and split <= 1e-5,
bfloat16 <= 3e-3; bfloat16 and split also against the float64 product of
the bfloat16-rounded operands (<= 1e-5), which pins round-to-nearest-even.
The 4096^3 case is the benchmark's launch configuration.
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

KINDS = {"f32": U.UPIR_BODY_MATMUL_F32, "bf16": U.UPIR_BODY_MATMUL_BF16, "split": U.UPIR_BODY_MATMUL_SPLIT3}
TOL = {"f32": 1e-5, "bf16": 3e-3, "split": 1e-5}


def note(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    U.lib()
    s = torch.cuda.Stream()
    prev = torch.cuda.current_stream()
    torch.cuda.set_stream(s)  # torch's work and the library's are ordered on one stream
    c = H.Context(0, stream=s)
    yield c
    c.close()
    torch.cuda.set_stream(prev)


def run_mm(ctx, kind, A, B, sched=None, spmd=None):
    M, K = A.shape
    N = B.shape[1]
    tA = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    tB = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    tC = torch.full((M, N), float("nan"), device="cuda")
    args = U.upir_matmul_args(tA.data_ptr(), tB.data_ptr(), tC.data_ptr(), K, K, N, N, None, 0)
    lp = ctx.loop(KINDS[kind], args, [(0, M, 1), (0, N, 1)], sched)
    variant = ctx.resolve(lp, spmd)[2]
    ctx.launch(lp, spmd)
    ctx.sync()
    out = tC.cpu().numpy()
    ctx.free(lp)
    return out, U.VARIANTS[variant]


@pytest.mark.parametrize("kind", ["f32", "bf16", "split"])
@pytest.mark.parametrize("M,N,K", [(256, 256, 64), (300, 260, 136), (32, 64, 8), (513, 129, 72)])
def test_mfma_integer_exact(ctx, kind, M, N, K):
    note(f"mfma int {kind} {M}x{N}x{K}")
    rng = np.random.default_rng(M + N + K)
    A = rng.integers(-2, 3, (M, K)).astype(np.float32)
    B = rng.integers(-2, 3, (K, N)).astype(np.float32)
    got, variant = run_mm(ctx, kind, A, B)
    # the float32 MFMA tiles load B rows as 16-byte vectors: N % 4 != 0 takes the generic kernel
    assert variant == ("generic" if kind == "f32" and N % 4 else "matmul_mfma")
    assert np.array_equal(got.astype(np.float64), bodies.matmul(A, B))


@pytest.mark.parametrize("kind", ["f32", "bf16", "split"])
@pytest.mark.parametrize("M,N,K,tile,units", [(384, 320, 256, None, None), (640, 512, 512, (256, 256), 512),
                                              (640, 512, 512, (128, 128), 256), (640, 512, 512, (256, 256), 256),
                                              (520, 300, 200, (256, 256), 256), (257, 513, 72, (256, 256), 256)])
def test_mfma_normal_parity(ctx, kind, M, N, K, tile, units):
    """Ragged shapes cover partial tiles in both dimensions and a k tail (K not
    a multiple of the 64-wide k step of the 256 x 256 four-wavefront tile)."""
    if kind == "f32" and tile == (256, 256):
        tile, units = (256, 128), 512
    note(f"mfma normal {kind} {M}x{N}x{K} tile={tile}")
    A = synth.normal(31, 0, M * K).reshape(M, K)
    B = synth.normal(31, 1, K * N).reshape(K, N)
    sched = H.make_sched(U.UPIR_SCHED_STATIC, tile=tile) if tile else None
    spmd = H.make_spmd(0, units) if units else None
    got, variant = run_mm(ctx, kind, A, B, sched, spmd)
    # the float32 MFMA tiles load B rows as 16-byte vectors: N % 4 != 0 takes the generic kernel
    assert variant == ("generic" if kind == "f32" and N % 4 else "matmul_mfma")
    C64 = bodies.matmul(A, B)
    assert bodies.frob_rel(got, C64) <= TOL[kind]
    if kind == "bf16":
        assert bodies.frob_rel(got, bodies.matmul_bf16(A, B)) <= 1e-5
    if kind == "split":
        assert bodies.frob_rel(got, bodies.matmul_split3(A, B)) <= 1e-5


def test_mfma_chunked_team_schedule(ctx):
    # tiles dealt to 3 teams in chunks of 2 tiles: same C
    A = synth.normal(32, 0, 520 * 264).reshape(520, 264)
    B = synth.normal(32, 1, 264 * 392).reshape(264, 392)
    got, variant = run_mm(ctx, "bf16", A, B, H.make_sched(U.UPIR_SCHED_STATIC_CHUNK, 2, tile=(128, 128)),
                          H.make_spmd(3, 256))
    assert variant == "matmul_mfma"
    assert bodies.frob_rel(got, bodies.matmul_bf16(A, B)) <= 1e-5


@pytest.mark.parametrize("kind", ["bf16", "split"])
@pytest.mark.parametrize("M,N,K,teams,chunked", [(512, 768, 96, 2, False), (512, 512, 128, 3, True),
                                                 (640, 520, 160, 2, False), (768, 256, 32, 2, True)])
def test_wide_tile_teams_with_several_tiles(ctx, kind, M, N, K, teams, chunked):
    """The four-wavefront 256 x 256 tile when a team computes several tiles one
    after another (the load ring restarts per tile), with odd and even numbers
    of 32-wide k steps, whole and partial tiles."""
    note(f"wide tile {kind} {M}x{N}x{K} teams={teams} chunked={chunked}")
    A = synth.normal(33, 0, M * K).reshape(M, K)
    B = synth.normal(33, 1, K * N).reshape(K, N)
    sched = (H.make_sched(U.UPIR_SCHED_STATIC_CHUNK, 1, tile=(256, 256)) if chunked
             else H.make_sched(U.UPIR_SCHED_STATIC, tile=(256, 256)))
    got, variant = run_mm(ctx, kind, A, B, sched, H.make_spmd(teams, 256))
    assert variant == "matmul_mfma"
    ref = bodies.matmul_bf16(A, B) if kind == "bf16" else bodies.matmul_split3(A, B)
    assert bodies.frob_rel(got, ref) <= 1e-5
    assert bodies.frob_rel(got, bodies.matmul(A, B)) <= TOL[kind]


@pytest.mark.parametrize("kind", ["f32", "bf16", "split"])
def test_mfma_full_size_4096(ctx, kind):
    n = 4096
    note(f"mfma 4096^3 {kind}")
    A = synth.normal(12345, 0, n * n).reshape(n, n)
    B = synth.normal(12345, 1, n * n).reshape(n, n)
    got, variant = run_mm(ctx, kind, A, B)
    assert variant == "matmul_mfma"
    # normwise error on a block of 512 full rows (every column, every k)
    rows = slice(1792, 2304)
    C64 = bodies.matmul(A[rows], B)
    err = bodies.frob_rel(got[rows], C64)
    note(f"  normwise error {err:.3e}")
    assert err <= TOL[kind]
    for (i, j) in [(0, 0), (4095, 4095), (1234, 3071), (4095, 0)]:
        ref = bodies.matmul_entry(A, B, i, j)
        scale = float(np.abs(A[i].astype(np.float64)) @ np.abs(B[:, j].astype(np.float64)))
        assert abs(got[i, j] - ref) <= 8 * TOL[kind] * scale


@pytest.mark.parametrize("kind", ["f32", "bf16", "split"])
def test_empty_reduction_dimension_gives_zero(ctx, kind):
    """K = 0: every entry of C is the empty sum, 0."""
    M, N = 64, 96
    tA = torch.zeros(M, 4, device="cuda")
    tB = torch.zeros(4, N, device="cuda")
    tC = torch.full((M, N), float("nan"), device="cuda")
    args = U.upir_matmul_args(tA.data_ptr(), tB.data_ptr(), tC.data_ptr(), 0, 4, N, N, None, 0)
    lp = ctx.loop(KINDS[kind], args, [(0, M, 1), (0, N, 1)])
    ctx.launch(lp)
    ctx.sync()
    assert (tC.cpu().numpy() == 0).all()
    ctx.free(lp)


@pytest.mark.parametrize("kind", ["f32", "bf16"])
def test_empty_output_writes_nothing(ctx, kind):
    tA = torch.ones(8, 8, device="cuda")
    tC = torch.full((8, 8), -3.0, device="cuda")
    args = U.upir_matmul_args(tA.data_ptr(), tA.data_ptr(), tC.data_ptr(), 8, 8, 8, 8, None, 0)
    lp = ctx.loop(KINDS[kind], args, [(0, 0, 1), (0, 8, 1)])
    ctx.launch(lp)
    ctx.sync()
    assert (tC.cpu().numpy() == -3.0).all()
    ctx.free(lp)
