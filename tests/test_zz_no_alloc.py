"""The entry point that allocates nothing (disc_embed_masks_noalloc) against
disc_embed_masks_ex on the same frames: outputs, statuses and pooled features
identical bit for bit (same kernels), on calls in a row whose second input is
smaller than the first, so a result never depends on what an earlier call
left in the shared scratch array."""
import numpy as np
import pytest

import disc_inputs as di
from gpu_common import COS_FP32, check_embeddings, dev_proj, frame_input, oracle_frame, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    t = torch()
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_03935_amd as disc

    disc.load()
    return disc


def _same(gpu, fr, proj, pooled, what):
    x = frame_input(fr)
    want = gpu.embed_frames([x], proj, pooled=pooled)[0]
    got = gpu.embed_masks_noalloc(x, proj, pooled=pooled)
    torch().cuda.synchronize()
    assert np.array_equal(got.status.cpu().numpy(), want.status.cpu().numpy()), f"{what}: status"
    assert np.array_equal(got.out.cpu().numpy(), want.out.cpu().numpy()), f"{what}: embeddings differ"
    if pooled:
        assert np.array_equal(got.pooled.cpu().numpy(), want.pooled.cpu().numpy()), f"{what}: pooled differ"
    return got


def test_noalloc_equals_embed_masks_ex(gpu):
    wl2 = di.workload("cfg2")
    fr = wl2.frames[0]
    p32 = dev_proj(wl2.proj, "f32")
    print("noalloc: cfg2 frame, 128 masks, FP32", flush=True)
    got = _same(gpu, fr, p32, True, "cfg2 FP32")
    check_embeddings(got.out.cpu().numpy(), got.status.cpu().numpy(), oracle_frame(fr, wl2.proj, "f32", idx=None),
                     COS_FP32, "noalloc cfg2")
    # second call, smaller: the 8 masks of a 336x336 frame
    wl1 = di.workload("cfg1")
    f1 = wl1.frames[0]
    print("noalloc: cfg1 frame, 8 masks, FP32", flush=True)
    _same(gpu, f1, dev_proj(wl1.proj, "f32"), False, "cfg1 FP32")
    # BF16 operands, then smaller again
    wl3 = di.workload("cfg3", frames=2)
    pb = dev_proj(wl3.proj, "bf16")
    print("noalloc: cfg3 frames 0-1, BF16", flush=True)
    _same(gpu, wl3.frames[0], pb, True, "cfg3 frame 0 BF16")
    small = di.Frame(wl3.frames[1].tokens, wl3.frames[1].bits[:5].copy(), wl3.frames[1].h, wl3.frames[1].w)
    _same(gpu, small, pb, False, "cfg3 frame 1, 5 masks, BF16")


def test_noalloc_rejects_workspace_and_oversize(gpu):
    import ctypes

    fr = di.workload("cfg1").frames[0]
    x = frame_input(fr)
    proj = dev_proj(di.workload("cfg1").proj, "f32")
    opts = gpu.make_options()
    buf = torch().empty(1 << 20, dtype=torch().uint8, device="cuda")
    opts.workspace = ctypes.c_void_p(buf.data_ptr())
    opts.workspace_bytes = 1 << 20
    with pytest.raises(gpu.DiscError):
        gpu.embed_masks_noalloc(x, proj, options=opts)
