"""The packed encoder and decode tables on the GPU (adgi_pack_channel, the
ones the packed blend uses) against the oracle's exact eq. rgbEnc, bit for
bit: at the binary32 values on both sides of every code boundary of the four
channels, and at random, zero, negative, tiny and huge values (needs an
MI355X)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

CHANNELS = [(0, 5.0, 15.0, 9), (1, 5.0, 15.0, 8), (2, 5.0, 15.0, 13), (3, 8.0, 20.0, 13)]


def _boundary_values(beta, gamma, bits):
    """T_k (first binary32 of code k) and the value below it, k = 1..qmax.
    The oracle's decoded value D_k is t_k rounded to nearest, so T_k is D_k
    or the next binary32."""
    qmax = (1 << bits) - 1
    out = []
    for k in range(1, qmax + 1):
        d = np.float32(oracle.pack_decode(k, beta, gamma, bits))
        t = d if oracle.pack_encode(float(d), beta, gamma, bits) == k else np.nextafter(d, np.float32(np.inf))
        out += [t, np.nextafter(t, np.float32(0.0))]
    return np.array(out, np.float32)


@pytest.mark.parametrize("channel,beta,gamma,bits", CHANNELS)
def test_device_codes_equal_the_exact_encoding(channel, beta, gamma, bits):
    import torch
    import paper_2301_05125_amd as adgi
    rng = np.random.default_rng(100 + channel)
    vals = np.concatenate([
        _boundary_values(beta, gamma, bits),
        np.exp(rng.uniform(np.log(1e-7), np.log(3e3), 200000)).astype(np.float32),
        np.array([0.0, -0.0, -1.0, 1e-40, 1e-30, 3.0e38, np.inf], np.float32),
    ]).astype(np.float32)
    codes, dec = adgi.pack_channel(torch.from_numpy(vals).cuda(), channel)
    torch.cuda.synchronize()
    codes = codes.cpu().numpy().astype(np.int64)
    dec = dec.cpu().numpy()
    ref = np.array([oracle.pack_encode(float(v), beta, gamma, bits) for v in vals], np.int64)
    bad = np.flatnonzero(codes != ref)
    assert bad.size == 0, [(float(vals[i]), int(codes[i]), int(ref[i])) for i in bad[:8]]
    qs = np.unique(ref)
    table = {int(q): np.float32(oracle.pack_decode(int(q), beta, gamma, bits)) for q in qs}
    want = np.array([table[int(q)] for q in ref], np.float32)
    assert np.array_equal(dec.view(np.uint32), want.view(np.uint32))
    # every code of the channel occurs (each boundary pair straddles one)
    assert qs.size == (1 << bits)
