"""The device filler of B reproduces the host generator bit for bit (sampled rows)."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbf,naux,dtype", [(24, 96, "f64"), (77, 51, "bf16"), (500, 2000, "bf16"),
                                            (1200, 4800, "bf16")])
def test_device_fill_matches_host(nbf, naux, dtype):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import synth.device as sdev
    key = synth.stream_key(synth.BASE_SEED + 3, 2)
    rows = [0, naux // 2, naux - 1]
    for p in rows:
        out = torch.empty((1, nbf, nbf), dtype=torch.bfloat16 if dtype == "bf16" else torch.float64, device="cuda")
        sdev.fill_b(out, key, nbf, naux, p)
        host = synth.b_chunk(key, nbf, naux, p, p + 1, dtype)
        if dtype == "bf16":
            bits = out.view(torch.int16).cpu().numpy().view(np.uint16)
            assert np.array_equal(bits, synth.f64_to_bf16_bits(host))
        else:
            assert np.array_equal(out.cpu().numpy(), host)
