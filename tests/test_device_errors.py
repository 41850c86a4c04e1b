"""Error paths that need no GPU: without a usable HIP device the library's create calls fail with
RCELL_ERR_DEVICE (-7) and a message naming the failed HIP call, leave nothing behind, and can be
called again with the same result.  (On a machine with a GPU the same code paths are exercised by
the injected allocation failures of the GPU tests.)"""
import pytest

from synth import configs


def _gpu_present():
    import torch
    return torch.cuda.device_count() > 0


pytestmark = pytest.mark.skipif(_gpu_present(), reason="needs a machine without a usable GPU")


def test_create_without_a_device_reports_a_device_error():
    from paper_1902_09171_amd import rcell, rsur
    rcell.load()
    for _ in range(2):
        with pytest.raises(rcell.RCellError) as e:
            rcell.RCellBatch(configs.kg_params(), [configs.kg_cell([20] * 10, 1)])
        assert e.value.code == -7 and "hipStreamCreate" in str(e.value)
    # argument errors are still reported as such, before any device call
    with pytest.raises(rcell.RCellError) as e:
        rcell.RCellBatch(dict(configs.kg_params(), dt=-1.0), [configs.kg_cell([20] * 10, 1)])
    assert e.value.code == -1
    with pytest.raises(rcell.RCellError) as e:
        rsur.Surrogate(din=8, width=16, depth=1, dout=2, ensemble=2, max_batch=64)
    assert e.value.code == -7 and "device" in str(e.value)
