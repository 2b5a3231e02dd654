"""Device decoder and the capped-iteration quality study on the GPU."""
import numpy as np
import pytest

import oracle
import synth
from stream_cases import huffman_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2604_18801_amd as pcc
    c = pcc.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("m_bits,mode", [(8, "vp"), (16, "hf"), (32, "sc")])
def test_device_decoder_equals_host_decoders(ctx, m_bits, mode):
    import paper_2604_18801_amd as pcc
    w = synth.cosmology(24, seed=21, xi=0.05)
    print("case decode_device", m_bits, mode, flush=True)
    stream, _, _ = ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode=mode, box=w.box,
                               m_bits=m_bits, max_iters=30)
    x_dev = ctx.decode_device(stream, _dev(w.recon)).cpu().numpy()
    np.testing.assert_array_equal(x_dev, pcc.decode(stream, w.recon))
    np.testing.assert_array_equal(x_dev, oracle.decode(stream, w.recon))


def test_device_decoder_of_oracle_stream(ctx):
    w = synth.plain_blobs(6000, seed=22)
    ref = oracle.correct(w.orig, w.recon, w.b, w.xi, mode="hf")
    x_dev = ctx.decode_device(ref.stream, _dev(w.recon)).cpu().numpy()
    np.testing.assert_array_equal(x_dev, oracle.decode(ref.stream, w.recon))


def test_device_decoder_on_hand_assembled_huffman_stream(ctx):
    """Two chunks (4 symbols, then 2) decoded by their own threads from the
    chunk starts, codes of 1 to 3 bits."""
    import paper_2604_18801_amd as pcc
    rec = np.array([[1.0, 2.0, 3.0, 4.0], [0.5] * 4, [-1.0] * 4], dtype=np.float32)
    stream, step, offset, codes = huffman_stream([0, 9])
    x = ctx.decode_device(stream, _dev(rec)).cpu().numpy()
    expect = rec.copy()
    for a in range(3):
        for k, pid in enumerate((0, 3)):
            expect[a, pid] = np.float32(float(rec[a, pid]) + codes[a][k] * step - offset)
    np.testing.assert_array_equal(x, expect)
    np.testing.assert_array_equal(pcc.decode(stream, rec), expect)


@pytest.mark.parametrize("starts,lengths", [([0, 8], (1, 2, 3, 3)), ([0, 10], (1, 2, 3, 3)),
                                            ([0, 12], (1, 2, 3, 3)), ([0, 9], (1, 1, 3, 3))])
def test_decoders_reject_corrupt_huffman_data(ctx, starts, lengths):
    """A chunk start that the codes do not reach, one past the bitstream, or
    code lengths that no prefix code has."""
    import paper_2604_18801_amd as pcc
    rec = np.zeros((3, 4), np.float32)
    stream, *_ = huffman_stream(starts, lengths)
    with pytest.raises(pcc.PccError):
        ctx.decode_device(stream, _dev(rec))
    with pytest.raises(pcc.PccError):
        pcc.decode(stream, rec)


def test_quality_study_rows(ctx):
    from paper_2604_18801_amd import quality
    w = synth.cosmology(32, seed=23, xi=0.05)
    print("case quality study cosmology32", flush=True)
    rows = list(quality.study(ctx, w, modes=("hf",), caps=(0, 1, None)))
    raw, capped, full = rows
    assert raw["mode"] == "none" and raw["membership_errors"] > 0 and raw["ari"] < 1.0
    assert full["status"] == 0 and full["membership_errors"] == 0
    assert full["ari"] == 1.0 and full["mwm_iou"] == 1.0 and full["hmf_rel_err_max"] == 0.0
    assert capped["iters"] == 1 and full["box_violations"] == 0 and capped["box_violations"] == 0
