"""ig_batch_progress_noalloc on the GPU: the entry point that allocates
nothing (its table and gather output live in a fixed device array) must
report exactly what ig_batch_progress reports, on two calls in a row, the
second over fewer contexts, through the C ABI."""
import pytest

from paper_2503_10516_amd import binding as B
from paper_2503_10516_amd import streams as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def test_progress_noalloc_equals_progress():
    streams = [S.stencil_1d(n=512, tasks=40), S.nbody_example(), S.random_small(3), S.random_small(9),
               S.growing(width=64, steps=24, devices=4, queue_cap=5),
               S.stencil_2d(side=256, tasks=30, nodes=2, devices=4, chunks=16)]
    print(f"[gpu] no-alloc progress over {len(streams)} contexts", flush=True)
    ctxs = []
    for s in streams:
        ctx = B.make_context(s)
        ctx.record(s)
        ctxs.append(ctx)
    # a windowed launch leaves the contexts at different points
    B.batch_flush(ctxs, window=25)
    for sub in (ctxs, ctxs[2:4]):
        want = B.batch_progress(sub)
        got = B.batch_progress(sub, noalloc=True)
        assert want.shape == got.shape == (len(sub), 6)
        assert (want == got).all(), (want, got)
        assert (want[:, 5] > 0).all()
    # and after the analysis has finished
    B.batch_flush(ctxs)
    for sub in (ctxs, ctxs[:1]):
        want = B.batch_progress(sub)
        got = B.batch_progress(sub, noalloc=True)
        assert (want == got).all(), (want, got)
        assert (got[:, 3] == 1).all()
    for c in ctxs:
        c.close()
