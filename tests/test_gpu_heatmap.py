"""The weighted similarity heat-map of text queries over a frame's patches
(disc_query_heatmap) against the FP64 oracle: heat[j][p] = D_p cos(t_j, f_p^T P)
for FP32, BF16 and FP8 tokens, a ragged patch grid, zero and degenerate
queries.  Bar: |got - want| <= 3e-5 * max_p D_p (FP32 arithmetic over
K = C and K = E, both near 1e-6 relative)."""
import numpy as np
import pytest

import disc_inputs as di
import oracle
from gpu_common import dev_proj, dev_tokens, torch

pytestmark = pytest.mark.gpu

TOL = 3e-5


@pytest.fixture(scope="module")
def gpu():
    t = torch()
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_03935_amd as disc

    disc.load()
    return disc


def _texts(seed, q, e, dtype, f64, P64):
    """q - 2 Gaussian queries, one equal to a projected token, one zero."""
    t, _ = di.normal_rows(seed, q, e, "f32")
    t = t.astype(np.float64)
    t[0] = f64[7] @ P64
    t[-1] = 0.0
    vals, _ = di.quantize(t, dtype)
    dec = oracle.decode_tokens(vals, dtype) if dtype == "bf16" else vals.astype(np.float64)
    return vals, dec


@pytest.mark.parametrize("name,tdtype,pdtype,h,w,patch,C,E", [
    ("cfg2 grid, FP32", "f32", "f32", 480, 640, 16, 1024, 768),
    ("ragged grid, BF16", "bf16", "bf16", 200, 264, 16, 256, 384),
    ("structured, FP8 tokens", "f8", "bf16", 480, 640, 16, 512, 256),
])
def test_heatmap_vs_oracle(gpu, name, tdtype, pdtype, h, w, patch, C, E):
    print(f"heatmap: {name}", flush=True)
    gh, gw = -(-h // patch), -(-w // patch)
    if tdtype == "f8":
        tok = di.tokens_structured(C + E, gh, gw, C, "f8", patch)
    else:
        tok = di.tokens_normal(C + E + gh, gh, gw, C, tdtype, patch)
    P = di.projection(C + 3, C, E, pdtype)
    f64 = oracle.decode_tokens(tok.data, tok.dtype, tok.scale).reshape(gh * gw, C)
    P64 = oracle.proj_to_f64(P, pdtype)
    text, text64 = _texts(E + 1, 21, E, "bf16" if pdtype == "bf16" else "f32", f64, P64)
    want = oracle.query_heatmap(f64, P64, text64)
    data, scale = dev_tokens(tok)
    tt = torch().from_numpy(np.ascontiguousarray(text))
    tt = (tt.view(torch().int16).cuda().view(torch().bfloat16) if text.dtype == np.uint16 else tt.cuda())
    got = gpu.query_heatmap(data, dev_proj(P, pdtype), tt, patch, scale).cpu().numpy().reshape(21, gh * gw)
    D = oracle.token_stats(f64)[2]
    err = np.abs(got.astype(np.float64) - want).max()
    assert err <= TOL * D.max(), f"{name}: max error {err:.3e} (max D {D.max():.3f})"
    assert not got[-1].any(), "zero text must give a zero row"
    assert np.all(np.abs(got) <= D[None, :] * (1 + 1e-5) + 1e-6)
    # the query equal to a projected token scores D_7 on that patch
    assert abs(got[0, 7] - D[7]) <= TOL * D.max()


def test_heatmap_two_valued(gpu):
    """A two-valued map (k patches u, the rest v): the GPU heat-map follows
    the oracle, and a query along the projected u scores D_u on the u
    patches.  (A constant map is 0/0 in Eq. 1, regularised by eps: FP32
    residuals of order eps make D there meaningless in FP32, so it is pinned
    on the oracle only.)"""
    gh, gw, C, E = 9, 11, 128, 128
    G = gh * gw
    rng = np.random.default_rng(12)
    u, v = rng.normal(size=C), rng.normal(size=C)
    vals = np.tile(v, (G, 1))
    idx = rng.choice(G, size=20, replace=False)
    vals[idx] = u
    tok = di.tokens_from_values(vals.reshape(gh, gw, C), "f32", 16)
    data, _ = dev_tokens(tok)
    P = di.projection(5, C, E, "f32")
    f64 = vals.astype(np.float32).astype(np.float64)
    P64 = P.astype(np.float64)
    t = np.stack([f64[idx[0]] @ P64, rng.normal(size=E)]).astype(np.float32)
    got = gpu.query_heatmap(data, dev_proj(P, "f32"), torch().from_numpy(t).cuda(), 16).cpu().numpy().reshape(2, G)
    want = oracle.query_heatmap(f64, P64, t.astype(np.float64))
    D = oracle.token_stats(f64)[2]
    assert np.abs(got - want).max() <= TOL * D.max()
    assert np.allclose(got[0, idx], D[idx], rtol=1e-5)
