"""The serving loop on the GPU: every result equals the frame processed alone
(bit for bit), with and without graph replay, under concurrent submitters;
a sample is also checked against the oracle."""
import threading

import numpy as np
import pytest

import disc_inputs as di
from gpu_common import COS_LOWP, check_embeddings, dev_proj, frame_input, oracle_frame, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def disc():
    t = torch()
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_03935_amd as d

    d.load()
    return d


@pytest.fixture(scope="module")
def stream_frames():
    counts = di.poisson_counts(di.frame_seed(4, 997), 12, 80.0, 1, 300)
    frames = []
    for i in range(12):
        big = i % 3 == 2
        h, w = (720, 1280) if big else (480, 640)
        frames.append(di.make_frame(4, 500 + i, h, w, int(counts[i]), 16, 1024, "bf16"))
    P = di.projection(di.frame_seed(4, 999), 1024, 768, "bf16")
    return frames, P


@pytest.mark.parametrize("use_graph", [True, False])
def test_server_matches_frames_alone(disc, stream_frames, use_graph):
    frames, P = stream_frames
    proj = dev_proj(P, "bf16")
    ins = [frame_input(f) for f in frames]
    alone = [disc.embed_frames([x], proj, quality=True)[0] for x in ins]
    torch().cuda.synchronize()
    with disc.Server(proj, tok_dtype=disc.DISC_BF16, c=1024, max_frames=4, max_masks=600, lanes=2,
                     use_graph=use_graph, mem_budget=8 << 30) as srv:
        results = [None] * len(ins)
        lock = threading.Lock()

        def producer(k):
            for i in range(k, len(ins), 3):
                t, out = srv.submit_frame(ins[i], quality=i % 2 == 0)  # half ask for dbar / area
                with lock:
                    results[i] = (t, out)

        th = [threading.Thread(target=producer, args=(k,)) for k in range(3)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        for i, (t, out) in enumerate(results):
            assert srv.wait(t) == 0, f"frame {i} failed"
        st = srv.stats()
        assert st["completed"] == len(ins) and st["failed"] == 0
        for i, (t, out) in enumerate(results):
            a, b = alone[i].out.cpu().numpy(), out.out.cpu().numpy()
            assert np.array_equal(a, b), f"frame {i}: served result differs from the frame alone"
            assert np.array_equal(alone[i].status.cpu().numpy(), out.status.cpu().numpy())
            if i % 2 == 0:
                assert np.array_equal(alone[i].dbar.cpu().numpy(), out.dbar.cpu().numpy()), f"frame {i}: dbar"
                assert np.array_equal(alone[i].area.cpu().numpy(), out.area.cpu().numpy()), f"frame {i}: area"
        for i in (0, 2):
            ref = oracle_frame(frames[i], P, "bf16")
            check_embeddings(results[i][1].out.cpu().numpy(), results[i][1].status.cpu().numpy(), ref, COS_LOWP,
                             f"served frame {i}")
        print(f"graph={use_graph}: {st['batches']} batches, mean {st['mean_batch_frames']:.2f} frames, "
              f"p50 {st['p50_ms']:.3f} ms p99 {st['p99_ms']:.3f} ms")


def test_server_graph_replays_many_batches(disc, stream_frames):
    """Replays of one captured graph with changing batch contents, interleaved
    with eager work on the default stream; every replay matches eager."""
    frames, P = stream_frames
    proj = dev_proj(P, "bf16")
    ins = [frame_input(f) for f in frames[:6]]
    alone = [disc.embed_frames([x], proj)[0].out.cpu().numpy() for x in ins]
    with disc.Server(proj, tok_dtype=disc.DISC_BF16, c=1024, max_frames=2, max_masks=600, lanes=1, use_graph=True,
                     mem_budget=8 << 30) as srv:
        for rep in range(3):
            outs = [srv.submit_frame(x) for x in ins]
            for t, _ in outs:
                assert srv.wait(t) == 0
            torch().cuda.synchronize()
            _ = disc.embed_frames([ins[rep]], proj)  # eager work between replays
            torch().cuda.synchronize()
            for i, (_, o) in enumerate(outs):
                assert np.array_equal(o.out.cpu().numpy(), alone[i]), f"replay {rep} frame {i} differs"
