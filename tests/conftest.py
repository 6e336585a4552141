import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    config.addinivalue_line(
        "markers", "final_path: GPU test of the loop's in-place final network (library defaults)")


@pytest.fixture(autouse=True)
def _loop_down_to_the_base_tile(request):
    """GPU tests run the QuickMergesort loop down to the base tile
    (final_tile 8192), so that their small inputs exercise partition rounds;
    tests marked final_path keep the library defaults."""
    if request.node.get_closest_marker("gpu") is None or \
            request.node.get_closest_marker("final_path") is not None:
        yield
        return
    import torch
    if not torch.cuda.is_available():
        yield
        return
    from paper_1804_10062_amd import autotune, qms
    d = autotune.DEFAULTS
    qms.qms_set_tuning(d[0], d[1], d[2], d[3], 8192)
    yield
    qms.qms_set_tuning(*d)
