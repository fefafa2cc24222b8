"""Reader for the small text fixtures holding numbers printed in the thesis."""
from __future__ import annotations

import pathlib

import numpy as np

HERE = pathlib.Path(__file__).resolve().parent


def load(name: str) -> dict:
    blocks: dict = {}
    cur = None
    for raw in (HERE / name).read_text().splitlines():
        line = raw.split("#", 1)[0].strip() if not raw.lstrip().startswith("[") else raw.strip()
        if not line:
            continue
        if line.startswith("["):
            cur = line[1:line.index("]")]
            blocks[cur] = []
            continue
        blocks[cur].append([float(v) for v in line.split()])
    return {k: np.array(v, dtype=np.float64).squeeze() if len(v) == 1 else np.array(v, dtype=np.float64)
            for k, v in blocks.items()}
