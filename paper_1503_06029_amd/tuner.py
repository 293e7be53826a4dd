"""Autotuner for the dictionary / edge parameters of a batch class.

Every parameter choice gives the same output bytes (the split bit s, the
directory width p and the group limit only decide which cells are found by
streaming and which by look-up), so the tuner may pick freely by speed.  It
times each candidate with HIP events on the class's real data, checks that
the edge count does not change, and keeps the fastest, keyed by (words per
row, log2 of the row count); the table persists as JSON.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import binding as B

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_params.json")


def candidates(ell: int, n_rows: int):
    """A small grid over s (split bit), p (directory bits) and group limit."""
    lg = max(1, math.ceil(math.log2(max(n_rows, 2))))
    out = []
    for s in sorted({min(ell, v) for v in (32, 64, 96, ((lg + 16 + 31) // 32) * 32)}):
        for gmax in (32, 64):
            out.append(dict(split_bit=s, dir_bits=min(lg, 22, ell), group_max=gmax))
    return out


def key_of(words: int, n_rows: int) -> str:
    return f"w{words}_n{max(0, int(math.log2(max(n_rows, 1))))}"


class Tuner:
    def __init__(self, path: str = DEFAULT_TABLE):
        self.path = path
        self.table = {}
        if os.path.exists(path):
            with open(path) as f:
                self.table = json.load(f)

    def save(self):
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def params_for(self, words: int, n_rows: int) -> B.DictParams | None:
        e = self.table.get(key_of(words, n_rows))
        return B.cg_dict_params_default(**e) if e else None

    def tune_class(self, sb, reps: int = 3):
        """Time candidate parameters on SceneBatch `sb` (already uploaded)."""
        ell = sb.lay.ell
        best, best_ms, ref_E = None, float("inf"), None
        for cand in candidates(ell, sb.n_rows):
            sb.params = B.cg_dict_params_default(**cand)
            sb.dict_bytes = B.cg_dict_size(sb.n_rows, sb.lay, sb.params)
            if sb.dict_mem.numel() < sb.dict_bytes:
                sb.dict_mem = torch.empty(sb.dict_bytes, dtype=torch.uint8, device=sb.device)
            sb.ws_edges = None
            sb.run()
            sb.ensure_capacity() or sb.run()
            torch.cuda.synchronize()
            E = int(sb.nedges.item())
            if ref_E is None:
                ref_E = E
            assert E == ref_E, "parameters changed the edge count"
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(reps):
                sb.run()
            t1.record()
            torch.cuda.synchronize()
            ms = t0.elapsed_time(t1) / reps
            if ms < best_ms:
                best, best_ms = cand, ms
        self.table[key_of(sb.words, sb.n_rows)] = best
        sb.params = B.cg_dict_params_default(**best)
        sb.dict_bytes = B.cg_dict_size(sb.n_rows, sb.lay, sb.params)
        sb.ws_edges = None
        return best, best_ms
