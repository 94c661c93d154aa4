"""A small JSON cache of autotuner choices, so that a tile shape timed once
for a grid, precision and GPU model is reused by later runs.

The file is named by the ``path`` argument or the TEUK_TUNE_CACHE
environment variable; without either nothing is cached.  Entries map
"<gpu>|fp<prec>|<n_theta>x<n_rstar>|<kind>" to a list of ints.  Writes go
through a temporary file and a rename, so a reader never sees a torn file.
"""
from __future__ import annotations

import json
import os

ENV = "TEUK_TUNE_CACHE"


def cache_path(path=None):
    return path if path is not None else os.environ.get(ENV) or None


def key(gpu: str, prec: int, shape, kind: str) -> str:
    nth, nr = shape
    return f"{gpu}|fp{int(prec)}|{int(nth)}x{int(nr)}|{kind}"


def lookup(path, k):
    if not path or not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            v = json.load(f).get(k)
    except (OSError, ValueError):
        return None
    return [int(x) for x in v] if isinstance(v, list) else None


def store(path, k, value):
    if not path:
        return
    data = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                data = json.load(f)
        except (OSError, ValueError):
            data = {}
    data[k] = [int(x) for x in value]
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
