import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def _gpu_available() -> bool:
    try:
        import torch
        return bool(torch.cuda.is_available())
    except Exception:  # pragma: no cover
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU visible in this process")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


def load_golden_windows():
    """Parse tests/golden/hand_windows.txt into {name: (src, dst, expected)}."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "hand_windows.txt")
    out = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, packets, expected = [p.strip() for p in line.split("|")]
            src, dst = [], []
            if packets != "-":
                for pair in packets.split():
                    s, d = pair.split(",")
                    src.append(int(s))
                    dst.append(int(d))
            exp = [int(x) for x in expected.split()]
            assert len(exp) == 9
            out[name] = (np.array(src, dtype=np.uint32), np.array(dst, dtype=np.uint32),
                         np.array(exp, dtype=np.uint64))
    return out


def load_golden_batch():
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "hand_batch.txt")
    fields = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = [p.strip() for p in line.split("|")]
            fields[k] = v.split()
    wins = load_golden_windows()
    names = fields["windows"]
    offsets = np.array([int(x) for x in fields["offsets"]], dtype=np.int64)
    src = np.concatenate([wins[n][0] for n in names]).astype(np.uint32)
    dst = np.concatenate([wins[n][1] for n in names]).astype(np.uint32)
    expected = np.stack([wins[n][2] for n in names])
    return src, dst, offsets, expected
