"""Autotuner cache: the fastest launch variant per (GPU architecture, geometry, batch).

The library times its own variants (shw_wfs_plan_autotune); this module
only remembers the answer in a JSON file so that later processes start with
the tuned variant.  Cache path: $SHW_AUTOTUNE_CACHE, else
~/.cache/shwfs/autotune.json.
"""
from __future__ import annotations

import json
import os

from . import shwfs


def cache_path() -> str:
    return os.environ.get("SHW_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "shwfs", "autotune.json"))


def key(arch: str, cfg, n_wfs: int, batch: int) -> str:
    return (f"{arch}|npx{cfg.npx}|fft{cfg.fft_n}|conv{cfg.conv_n}|det{cfg.det_n}|lgs{cfg.lgs}"
            f"|noise{int(bool(cfg.flags & 1))}|wfs{n_wfs}|batch{batch}")


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def tuned_variant(plan: "shwfs.WfsPlan", opd, slopes, arch: str, reps: int = 20, stream=None, retune=False):
    """Select the plan's launch variant from the cache, or time all variants and record the winner."""
    path = cache_path()
    k = key(arch, plan.cfg, plan.n_wfs, opd.shape[0])
    table = _load(path)
    if not retune and k in table and 0 <= table[k]["variant"] < plan.n_variants:
        plan.set_variant(table[k]["variant"])
        return table[k]
    best, ms = plan.autotune(opd, slopes, reps=reps, stream=stream)
    rec = {"variant": best, "ms_per_launch": ms}
    table[k] = rec
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return rec
