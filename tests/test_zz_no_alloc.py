"""unihenn_rotate_noalloc, the rotation for callers that cannot allocate,
against unihenn_rotate: bit for bit on two calls in a row (the second with a
smaller input, so it runs on what the first left in the shared scratch
array), both also equal to the CPU oracle's rotation; a rotation whose
workspace exceeds the fixed scratch size is refused and writes nothing."""
from __future__ import annotations

import numpy as np
import pytest

from tests.gpu_util import gpu_ctx_for, ocat, oracle_ring, random_ct

pytestmark = pytest.mark.gpu

RING = {"log_n": 14, "prime_bits": [60] + [40] * 7, "special_bits": 60, "log_scale": 40}
STEPS = 5


@pytest.fixture(scope="module")
def pair():
    ck = oracle_ring(RING)
    ctx = gpu_ctx_for(ck, RING)
    key_coeff = ck.rotation_key(STEPS)
    return ck, ctx, key_coeff, ctx.import_evk(key_coeff)


def test_rotate_noalloc_equals_rotate_twice_shrinking(pair):
    import torch
    ck, ctx, key_coeff, key = pair
    okey = ck.load_key(key_coeff)
    # first call: 8 limbs x 3 ciphertexts (~51 MB of scratch); second: 4 limbs x 1
    for nl, batch, seed in ((8, 3, 101), (4, 1, 102)):
        coeff = random_ct(ck, nl, seed, batch=batch)
        x = ctx.import_ct(coeff, 2.0 ** 40)
        ws = ctx.workspace(nl, batch)
        ref = ctx.rotate(x, STEPS, key, ws)
        out = ctx.empty_ct(batch, nl)
        out.data.fill_(-1)
        ctx.rotate_noalloc(x, STEPS, key, out)
        torch.cuda.synchronize()
        assert out.scale == ref.scale
        assert torch.equal(out.data, ref.data), (nl, batch)
        got = ctx.export_ct(out)
        for b in range(batch):
            exp = ck.rotate(ocat(coeff[b]), STEPS, okey).data
            assert np.array_equal(got[b], exp), (nl, batch, b)


def test_rotate_noalloc_refuses_past_the_scratch_size(pair):
    import torch
    import paper_2402_03060_amd as P
    ck, ctx, _, key = pair
    # 8 limbs x 4 ciphertexts need 4 * 130 rows of 128 KiB = 68 MB > 64 MiB
    nl, batch = 8, 4
    assert P.lib().unihenn_ks_workspace_size(ctx.h, nl, batch) > 64 << 20
    x = ctx.import_ct(random_ct(ck, nl, 103, batch=batch), 2.0 ** 40)
    out = ctx.empty_ct(batch, nl)
    out.data.fill_(7)
    torch.cuda.synchronize()
    with pytest.raises(P.UnihennError) as ei:
        ctx.rotate_noalloc(x, STEPS, key, out)
    assert ei.value.code == P.EINVAL and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((out.data == 7).all())
