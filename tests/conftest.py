import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _ensure_built():
    """Build what is not built yet: the generator, the CPU reference, the HIP library."""
    import synth
    import oracle
    if not os.path.exists(os.path.join(ROOT, "synth", "libsynth.so")):
        synth.build()
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build()
    if not os.path.exists(os.path.join(ROOT, "paper_1808_05056_amd", "libooc.so")):
        import importlib.util
        spec = importlib.util.spec_from_file_location("ooc_build", os.path.join(ROOT, "paper_1808_05056_amd", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()


_ensure_built()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running")
