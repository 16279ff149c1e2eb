import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running (large grids)")


@pytest.fixture(scope="session")
def O():
    import oracle
    oracle.lib()
    return oracle


# Measured parity errors (relative L2 per component against the reference of
# each test), printed as they are taken and, when PST_ERROR_LOG names a file,
# written there as JSON at the end of the session.
_ERRS = []


@pytest.fixture
def errlog(request):
    def record(label, errs, tol):
        errs = [float(e) for e in errs]
        _ERRS.append({"test": request.node.nodeid, "label": label, "rel_l2": errs, "tol": tol})
        print(f"[parity] {request.node.nodeid} {label}: " + " ".join(f"{e:.3e}" for e in errs)
              + f" (tol {tol:.0e})", flush=True)
        assert max(errs) < tol, (label, errs, tol)
    return record


def pytest_sessionfinish(session, exitstatus):
    path = os.environ.get("PST_ERROR_LOG")
    if path and _ERRS:
        import json
        with open(path, "w") as fh:
            json.dump(_ERRS, fh, indent=1)
