"""The LDS atomic microbenchmark (libkc_probe.so) does the work it is timed
for: every add lands (the words sum to the number of adds), and the OR kinds
run and report a positive time."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


@pytest.mark.parametrize("words_log2", [6, 12, 13, 15])
def test_probe_adds_all_land(words_log2):
    from paper_1712_03254_amd import probe
    from kc_cases import note
    note("case: probe adds, 2^%d words, 300 workgroups x 3 iterations" % words_log2)
    ops, ms, chk = probe.lds_atomics(probe.KCP_ADD, words_log2, iters=3, blocks=300)
    assert ops == 300 * 1024 * 3 * 8
    assert chk == ops
    assert ms > 0


def test_probe_or_kinds_run():
    from paper_1712_03254_amd import probe
    from kc_cases import note
    note("case: probe OR kinds, 2^13 words")
    for kind in (probe.KCP_OR, probe.KCP_OR_RTN):
        ops, ms, chk = probe.lds_atomics(kind, 13, iters=4, blocks=512)
        assert ms > 0 and 0 < chk
    rate = probe.lds_atomic_peak(probe.KCP_OR_RTN, 13, reps=1)
    note("or-with-return peak %.3g /s" % rate)
    assert rate > 1e10
