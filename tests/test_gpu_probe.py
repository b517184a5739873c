"""The MFMA-rate probe runs and reports a rate below the nominal dense INT8
peak (5.0 POP/s), and the residue products of an 8192 x 8192 x 1024 product
do not exceed it (the probe is their ceiling on this chip)."""
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2602_02549_amd as oz  # noqa: E402


def test_probe_rate_is_physical():
    announce("MFMA-rate probe")
    rc, ms, ops = oz.ozaki2_debug_mfma_probe(512)
    assert rc == oz.OK and ms > 0
    assert ops == torch.cuda.get_device_properties(0).multi_processor_count * 8 * 512 * 8 * 65536
    for changing in (1, 0):
        rc, ms, ops = oz.ozaki2_debug_mfma_probe(4096, changing)
        assert rc == oz.OK
        tops = ops / (ms * 1e-3) / 1e12
        assert 100.0 < tops < 5000.0 * 1.05, (changing, tops)
