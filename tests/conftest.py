import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


# Run the suite against another build of the library (the sanitized host
# build of tests/test_sanitized_host.py) when GIAMG_TEST_LIBRARY names one.
if os.environ.get("GIAMG_TEST_LIBRARY"):
    from paper_2512_15121_amd import giamg as _giamg
    _giamg.LIB_PATH = os.environ["GIAMG_TEST_LIBRARY"]
