import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def load_oracle_tables():
    """Oracle SOE tables written by tests/golden/make_oracle_tables.py."""
    with open(os.path.join(GOLDEN, "oracle_soe_tables.json")) as f:
        raw = json.load(f)["tables"]
    out = {}
    for k, t in raw.items():
        out[int(k)] = {
            "tau0": np.array(t["tau0_re"]) + 1j * np.array(t["tau0_im"]),
            "omega": np.array(t["omega_re"]) + 1j * np.array(t["omega_im"]),
            "E": t["E"], "Eprime": t["Eprime"], "sum_abs_omega": t["sum_abs_omega"],
        }
    return out


def load_paper_numbers():
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as f:
        return json.load(f)


@pytest.fixture(scope="session")
def otables():
    return load_oracle_tables()


@pytest.fixture(scope="session")
def paper():
    return load_paper_numbers()
