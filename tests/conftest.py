import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU run; enabled with ESQ_SLOW=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("ESQ_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow CPU pin; set ESQ_SLOW=1 to run")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)


def read_golden(name):
    """Rows of whitespace-separated ints/floats from tests/golden/<name>."""
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


def load_oracle_sample(name):
    """A stored oracle sample (tests/golden/make_oracle_samples.py): (meta,
    ns, k, parts), with the drawn n regenerated and checked."""
    import importlib.util
    path = os.path.join(ROOT, "tests", "golden", "make_oracle_samples.py")
    spec = importlib.util.spec_from_file_location("make_oracle_samples", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.load(name)
