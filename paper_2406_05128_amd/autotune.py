"""Persistent cache of chunk lengths chosen by the native autotuner (lp_plan_autotune).

One JSON object per file: {"<device>|M=<M>|B=<B>|T=<T>[|carry=<constraint>][|lib=<id>]":
{"chunk": L, "chained": bool, "ms": t}}.  The library id names the build the
choice was measured with, so a rebuilt library (other kernels) tunes afresh.
Writes go through a temporary file and an atomic rename.
"""
from __future__ import annotations

import json
import os
import tempfile
from typing import Optional


def cache_path() -> str:
    return os.environ.get("TVLP_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "tvlp", "autotune.json"))


def cache_key(device_name: str, M: int, B: int, T: int, carry: str = "grouped", lib: str = "") -> str:
    key = f"{device_name}|M={int(M)}|B={int(B)}|T={int(T)}"
    if carry != "grouped":
        key = f"{key}|carry={carry}"
    return f"{key}|lib={lib}" if lib else key


def _read(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def lookup(key: str) -> Optional[dict]:
    hit = _read(cache_path()).get(key)
    if isinstance(hit, dict) and isinstance(hit.get("chunk"), int) and hit["chunk"] > 0:
        return {"chunk": hit["chunk"], "chained": bool(hit.get("chained", False)), "ms": float(hit.get("ms", 0.0))}
    return None


def store(key: str, value: dict) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    data = _read(path)
    data[key] = {"chunk": int(value["chunk"]), "chained": bool(value.get("chained", False)),
                 "ms": float(value["ms"])}
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(path) or ".", suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
