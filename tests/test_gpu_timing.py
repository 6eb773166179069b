"""Kernel timing diagnostics through the C-ABI: sampled HIP-event timing of
the instrumented kernel classes."""
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_sampled_timing_counts_and_values():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_17494_amd import Context, make_iters, make_layout, make_params
    ctx = Context(0)
    try:
        _, d64 = synth.noisy_f32(40, 48, 0.1, 2)
        d0 = torch.tensor(d64, dtype=torch.float32, device="cuda:0")
        prm, lay = make_params(0.15, 10.0), make_layout(2, 2, 4, 4)
        sweeps, inner = 2, 9
        for every in (1, 4):
            ctx.timing_reset()
            ctx.timing(True, every=every)
            ctx.schwarz_solve(d0, prm, lay, make_iters(sweeps, inner))
            ctx.timing(False)
            t = ctx.timing_read()
            calls = sweeps * inner  # s1_update runs once per inner iteration
            assert t["s1_update"][0] == (calls + every - 1) // every
            for name, (n, ms, nbytes) in t.items():
                assert n >= 1 and ms > 0 and nbytes > 0, name
        with pytest.raises(ValueError):
            ctx.timing(True, every=0)
    finally:
        ctx.close()
