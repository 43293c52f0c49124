import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


_REPORT = {}


@pytest.fixture(scope="session")
def report():
    """Measured errors of the GPU parity tests; written to
    gpurun_out/parity_report.json (or $LM_REPORT) at the end of the session."""
    return _REPORT


def pytest_sessionfinish(session, exitstatus):
    if not _REPORT:
        return
    import json
    path = os.environ.get("LM_REPORT", os.path.join(ROOT, "gpurun_out", "parity_report.json"))
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump({"|".join(map(str, k)): v for k, v in sorted(_REPORT.items(), key=lambda kv: str(kv[0]))},
                  f, indent=1, default=float)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def pytest_collection_modifyitems(config, items):
    # GPU tests are skipped (not failed) when no GPU is present, so that
    # `-m "not gpu"` and a plain run both work on a CPU-only host.
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU available")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
