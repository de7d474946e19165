import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    oracle.build(force=False)
    yield


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    """Parse a golden fixture: '# ...' comments, 'NAME rows cols' blocks and
    'key values...' lines.  Returns dict of name -> ndarray or list of lists."""
    import numpy as np
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    i = 0
    while i < len(lines):
        parts = lines[i].split()
        if len(parts) == 3 and parts[1].isdigit() and parts[2].isdigit():
            r, c = int(parts[1]), int(parts[2])
            rows = [[float(x) for x in lines[i + 1 + q].split()] for q in range(r)]
            out[parts[0]] = np.array(rows, dtype=np.float64).reshape(r, c)
            i += 1 + r
        else:
            out.setdefault(parts[0], []).append(parts[1:])
            i += 1
    return out
