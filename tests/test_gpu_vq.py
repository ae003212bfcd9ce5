"""Decode of vector-quantised model attributes (veg_vq_decode) against the oracle, bit for
bit, and a model rendered from its decoded codebook against the oracle's render of the same
decoded model."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import compare_image, hip, image_pixels, luts_to_dev

pytestmark = pytest.mark.gpu


def _decode(idx, book, widths):
    V, R = hip()
    n = idx.shape[0]
    outs = [torch.empty((n,) if w == 1 else (n, w), dtype=torch.float32, device="cuda") for w in widths]
    V.veg_vq_decode(torch.as_tensor(idx).cuda(), torch.as_tensor(book).cuda(), outs)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("n,k,widths", [(100003, 4096, [3, 4]), (1, 1, [7]), (5000, 65536, [3, 1, 1, 1, 1]),
                                        (777, 300, [1, 2, 3, 4, 5, 1])])
def test_decode_is_bit_exact_including_out_of_range_indices(n, k, widths):
    rng = np.random.default_rng(n + k)
    dim = sum(widths)
    book = rng.standard_normal((k, dim)).astype(np.float32)
    idx = rng.integers(0, 65536, n).astype(np.uint16) if k < 65536 else rng.integers(0, k, n).astype(np.uint16)
    if k < 65536:
        idx[::3] = rng.integers(0, k, idx[::3].shape[0])   # mostly valid, some beyond the codebook
    got = _decode(idx, book, widths)
    ref = oracle.vq_decode(idx, book, widths)
    for g, r in zip(got, ref):
        assert g.shape == r.shape
        assert np.array_equal(g.view(np.uint32), r.view(np.uint32))


def test_empty_decode_is_a_no_op():
    V, R = hip()
    out = torch.full((0, 3), 5.0, device="cuda")
    V.veg_vq_decode(torch.zeros(0, dtype=torch.uint16).cuda(), torch.zeros((4, 3)).cuda(), [out])
    torch.cuda.synchronize()


def test_render_from_a_decoded_codebook_matches_oracle():
    """A 3000-Gaussian model with its shape (log-scales and quaternion) compressed to 256
    codewords: decoded on the GPU and rendered, against the oracle's render of the model
    the oracle decodes from the same codebook."""
    V, R = hip()
    w = synth.workload(1, n_override=3000, views_override=1, tfs_override=1, res_override=96)
    g = w.gaussians
    shape = np.concatenate([g.log_scales, g.quats], 1).astype(np.float32)
    idx, book = synth.vq_encode(np.random.default_rng(8), shape, 256, iters=3)
    ls, q = oracle.vq_decode(idx, book, [3, 4])
    gd = synth.Gaussians(g.means, ls, q, g.scalars, g.weights)
    dev = V.decode_vq_model(torch.as_tensor(g.means).cuda(), torch.as_tensor(g.scalars).cuda(),
                            torch.as_tensor(idx).cuda(), torch.as_tensor(book).cuda(),
                            None if g.weights is None else torch.as_tensor(g.weights).cuda())
    assert np.array_equal(dev.log_scales.cpu().numpy(), ls) and np.array_equal(dev.quats.cpu().numpy(), q)
    st = R.render(dev, [w.cameras[0]], luts_to_dev([w.tfs[0]]), w.opts)
    torch.cuda.synchronize()
    res, *_ = oracle.render_image(gd, w.cameras[0], w.tfs[0], w.opts)
    compare_image(image_pixels(st.image[0]), res)
