import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def read_sections(path):
    """Parse the [name] / key: value / matrix-block fixture format."""
    sections, cur, key = {}, None, None
    with open(path) as f:
        for raw in f:
            line = raw.rstrip("\n")
            if not line.strip() or line.lstrip().startswith("#"):
                continue
            if line.startswith("["):
                cur = sections.setdefault(line.strip()[1:-1], {})
                key = None
                continue
            if ":" in line and line.split(":")[0].strip() in (
                    "cite", "symbols", "points", "m", "r", "BT", "G", "AT"):
                k, v = line.split(":", 1)
                key = k.strip()
                v = v.strip()
                cur[key] = v if v else []
                continue
            cur[key].append(line.strip())
    return sections


def read_table(path):
    rows = []
    with open(path) as f:
        for raw in f:
            if not raw.strip() or raw.lstrip().startswith("#"):
                continue
            rows.append([c.strip() for c in raw.split("|")])
    return rows
