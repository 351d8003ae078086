import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line(
        "markers", "slow: long CPU oracle runs (full-size sampled parity)")


def ensure_library():
    """Build libtnrg.so when it is missing, loading the build script by path
    (the package itself cannot be imported before the library exists)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "_tnrg_build", os.path.join(ROOT, "paper_2603_03639_amd", "build.py"))
    B = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(B)
    if not os.path.exists(B.LIB_PATH):
        B.build()
    return B.LIB_PATH
