"""Autotuner for the dictionary / edge parameters of a batch class.

Every parameter choice gives the same output bytes (the edge path -- flip
and look-up or the O(n l) hash probes --, the split bit s, the directory
width p and the group limit only decide how each edge is found, the sort-key
width only how rows are ordered before full-row tie-breaking), so the
tuner may pick freely by speed.  It times each candidate with HIP events on
the class's real data (the whole class run: pack, dedup, dictionary, edges,
split), checks that the edge count does not change, and keeps the fastest,
keyed by (words per row, log2 of the row count); the table persists as
JSON.  Parameters are read back through the library's
cg_dict_params_tuned, which picks the nearest entry for a size.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import binding as B

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_params.json")


def candidates(ell: int, n_rows: int, tag_bits: int = 0):
    """A small grid over s (split bit) and the group limit; tag_bits leading
    bits that never differ inside a scene (a batch's scene tag) are skipped."""
    lg = max(1, math.ceil(math.log2(max(n_rows, 2))))
    splits = {tag_bits + d for d in (16, 32, 48, 64, 96, 128, 192, 256, 384)}
    splits.add(((lg + 16 + 31) // 32) * 32)
    out = []
    for s in sorted(v for v in splits if tag_bits < v < ell):
        for gmax in (32, 64):
            out.append(dict(split_bit=s, dir_bits=min(lg, 22, ell), group_max=gmax))
    # the O(n l) hash probes need no suffix order (split 0)
    out.append(dict(path=B.CG_PATH_HASH, split_bit=0, dir_bits=min(lg, 22, ell)))
    return out


def log2_rows(n_rows: int) -> int:
    return max(0, int(math.log2(max(n_rows, 1))))


def key_of(words: int, n_rows: int) -> str:
    return f"w{words}_n{log2_rows(n_rows)}"


class Tuner:
    def __init__(self, path: str | None = DEFAULT_TABLE):
        """path=None: an in-memory table (nothing read or written)."""
        self.path = path
        self.table = {}
        if path is not None and os.path.exists(path):
            with open(path) as f:
                self.table = json.load(f)

    def save(self):
        if self.path is None:
            return
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def entries(self):
        """The table as (words, log2 rows, DictParams) entries."""
        out = []
        for k, e in sorted(self.table.items()):
            w, n = k[1:].split("_n")
            out.append((int(w), int(n), B.cg_dict_params_default(**e)))
        return out

    def params_for(self, words: int, n_rows: int) -> B.DictParams | None:
        """The library's pick from the table for this class (the entry with
        these words and the nearest size), or None without such an entry."""
        ents = self.entries()
        if not any(w == words for w, _, _ in ents):
            return None
        lay = B.cg_batch_layout(32 * (words - 1))
        return B.cg_dict_params_tuned(ents, n_rows, lay)

    def tune_class(self, sb, reps: int = 2, tag_bits: int = 32):
        """Time candidate parameters on SceneBatch `sb` (already uploaded).
        A candidate whose first run is more than 3x slower than the best so
        far is dropped without further timing."""
        ell = sb.lay.ell
        best, best_ms, ref_E = None, float("inf"), None

        def timed_run():
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record()
            sb.run()
            t1.record()
            torch.cuda.synchronize()
            return t0.elapsed_time(t1)

        for cand in candidates(ell, sb.n_rows, tag_bits):
            sb.params = B.cg_dict_params_default(**cand)
            sb.dict_bytes = B.cg_dict_size(sb.n_rows, sb.lay, sb.params)
            if sb.dict_mem.numel() < sb.dict_bytes:
                sb.dict_mem = torch.empty(sb.dict_bytes, dtype=torch.uint8, device=sb.device)
            sb.ws_edges = None
            first = timed_run()
            if not sb.ensure_capacity():
                first = timed_run()
            E = int(sb.nedges.item())
            if ref_E is None:
                ref_E = E
            assert E == ref_E, "parameters changed the edge count"
            if first > 3 * best_ms:
                continue
            ms = min(timed_run() for _ in range(reps))
            if ms < best_ms:
                best, best_ms = cand, ms
        # then the sort-key width of the fused dedup + dictionary build, with
        # the best edge parameters (0: separate calls, automatic width)
        for kb in (32, 64, 96):
            cand = dict(best, key_bits=kb)
            sb.params = B.cg_dict_params_default(**cand)
            timed_run()
            assert int(sb.nedges.item()) == ref_E, "key width changed the edge count"
            ms = min(timed_run() for _ in range(reps))
            if ms < best_ms:
                best, best_ms = cand, ms
        self.table[key_of(sb.words, sb.n_rows)] = best
        sb.params = B.cg_dict_params_default(**best)
        sb.dict_bytes = B.cg_dict_size(sb.n_rows, sb.lay, sb.params)
        if sb.dict_mem.numel() < sb.dict_bytes:
            sb.dict_mem = torch.empty(sb.dict_bytes, dtype=torch.uint8, device=sb.device)
        sb.ws_edges = None
        return best, best_ms
