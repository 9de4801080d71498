"""Continuous-batching server on the GPU: with a budget small enough to force
admission waits and several launch slots in flight, every request's image is
bitwise the image of the same frame beamformed alone, and within the reduced-
precision tolerance of the oracle."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2203_14906_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pool():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2203_14906_amd import serve
    p = serve.FramePool(torch, "cuda", n_elements=(16, 32), n_samples=(256, 512), sides=(32, 48),
                        seed=77)
    yield p
    p.close()


def test_server_results_equal_alone_and_admission(pool):
    from paper_2203_14906_amd import serve
    reqs = serve.poisson_requests(4000.0, 0.08, len(pool.frames), seed=3)
    # a burst at the start: more simultaneous arrivals than the budget holds,
    # so admission waits do not depend on how fast the GPU drains the queue
    for r in reqs[:24]:
        r.arrival = reqs[0].arrival
    say("requests:", len(reqs))
    one = max(f.side * f.side * 4 + f.n_elements * f.n_samples * 2 for f in pool.frames)
    srv = serve.Server(torch, pool, slots=3, budget_bytes=3 * one, max_batch=8)
    st = srv.run(reqs, keep_images=True)
    torch.cuda.synchronize()
    summ = st.summary()
    say("batched:", summ)
    assert all(r.done >= r.arrival and r.status == "done" for r in reqs)
    assert st.admission_waits > 0, "the tiny budget should make requests wait"
    assert st.launches > 1
    for r in reqs:
        fr = pool.frames[r.frame]
        alone = fr.plan16.beamform(fr.rf16, r.order)
        torch.cuda.synchronize()
        assert torch.equal(alone, r.image), "request %d differs from its alone result" % r.rid
    # parity of a few requests against the oracle on the same stored values
    for r in reqs[:6]:
        fr = pool.frames[r.frame]
        w, d = ph.field_of_view(fr.n_elements, fr.n_samples)
        grid = ph.make_grid(fr.side, fr.side, w, d)
        ref = O.beamform(fr.rf16.cpu().numpy(), ph.Geometry(fr.n_elements), grid, r.order)
        g = r.image.cpu().numpy().astype(np.float64)
        err = np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300)
        say("request %d order %d rel L2 %.2e" % (r.rid, r.order, err))
        assert err <= 2e-3 and err <= 2e-5
    srv.close()


def test_plain_loop_and_overlap(pool):
    from paper_2203_14906_amd import serve
    reqs = serve.poisson_requests(3000.0, 0.05, len(pool.frames), seed=4)
    plain = serve.run_plain(torch, pool, reqs)
    say("plain:", plain.summary())
    assert plain.latencies_ms.min() >= 0
    reqs2 = serve.poisson_requests(20000.0, 0.02, len(pool.frames), seed=5)
    for r in reqs2[:96]:                      # a burst: launches queue up behind each other
        r.arrival = reqs2[0].arrival
    srv = serve.Server(torch, pool, slots=3, budget_bytes=32 << 30, max_batch=4)
    st = srv.run(reqs2)
    say("batched burst:", st.summary())
    assert st.max_inflight > 1
    srv.close()


def test_rejected_requests_leave_the_rest_intact(pool):
    from paper_2203_14906_amd import serve
    reqs = serve.poisson_requests(4000.0, 0.02, len(pool.frames), seed=6)
    reqs[2].order, reqs[5].frame = 7, len(pool.frames) + 3
    srv = serve.Server(torch, pool, slots=2, budget_bytes=32 << 30, max_batch=8)
    st = srv.run(reqs, keep_images=True)
    torch.cuda.synchronize()
    say("with rejections:", st.summary())
    assert st.rejected == 2 and reqs[2].status == reqs[5].status == "rejected"
    for r in reqs:
        if r.rid in (2, 5):
            assert r.image is None
            continue
        fr = pool.frames[r.frame]
        assert r.status == "done" and torch.equal(fr.plan16.beamform(fr.rf16, r.order), r.image)
    srv.close()


def test_server_with_mirror_pairs():
    """The serving pool with paired FP16 plans: batches mix pair kinds of
    several orders, and every request's image is still bitwise its frame's own
    paired launch; a few are checked against the oracle (sign-change pixels
    measured from the oracle's delay band)."""
    from paper_2203_14906_amd import hodmas, serve
    from sign_band import band_rel_l2
    p = serve.FramePool(torch, "cuda", n_elements=(16, 32), n_samples=(256, 512), sides=(32, 48),
                        seed=78, plain=False, mirror=True)
    assert all(fr.plan16.info().flags & hodmas.FLAG_MIRROR for fr in p.frames)
    reqs = serve.poisson_requests(4000.0, 0.06, len(p.frames), seed=6)
    for r in reqs[:24]:
        r.arrival = reqs[0].arrival
    srv = serve.Server(torch, p, slots=3, budget_bytes=32 << 30, max_batch=8)
    st = srv.run(reqs, keep_images=True)
    torch.cuda.synchronize()
    say("batched, mirror pairs:", st.summary())
    assert all(r.status == "done" for r in reqs)
    for r in reqs:
        fr = p.frames[r.frame]
        alone = fr.plan16.beamform(fr.rf16, r.order)
        torch.cuda.synchronize()
        assert torch.equal(alone, r.image), "request %d differs from its alone result" % r.rid
    for r in reqs[:6]:
        fr = p.frames[r.frame]
        w, d = ph.field_of_view(fr.n_elements, fr.n_samples)
        grid = ph.make_grid(fr.side, fr.side, w, d)
        err, flagged = band_rel_l2(r.image.cpu().numpy(), fr.rf16.cpu().numpy(), ph.Geometry(fr.n_elements),
                                   grid, r.order)
        say("request %d order %d rel L2 from the band %.2e (%d sign-change pixels)" % (r.rid, r.order, err, flagged))
        assert err <= 2e-5
    srv.close()
    p.close()
