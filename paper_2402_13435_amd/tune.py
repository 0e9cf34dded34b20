"""Autotune the library on this GPU for the standard synthetic workloads and
write the tuning table that searches load (JSON lines, one entry per batch
shape; see fr_tuning_save in include/fr.h).

    python -m paper_2402_13435_amd.tune --out paper_2402_13435_amd/tuning/gfx950.jsonl

Workloads: the 1,000,000 x 128 corpus of the FP32 configuration (vocabulary
4,096), FP32 with K = 100, BF16 with R = 100 and FP8 with R = 128 (the
rescoring depths the benchmark selects), batches of 1, 32, 256 and 1,024
queries.  Each shape is tuned on queries the benchmark does not time (the
tail of a 2,048-query batch of the same recipe).
"""
from __future__ import annotations

import argparse
import os
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True, help="tuning table to write (JSON lines)")
    ap.add_argument("--batches", default="1,32,256,1024")
    args = ap.parse_args()
    import datagen
    from paper_2402_13435_amd import Index
    c = datagen.corpus(datagen.CONFIGS["fp32"])
    df = datagen.doc_frequency(c.cfg, c.term_off, c.terms)
    pool = datagen.queries(c.cfg, df, n_queries=2048)
    sizes = [int(x) for x in args.batches.split(",")]
    lines = []
    for dtype, r in (("f32", 0), ("bf16", 100), ("fp8", 128)):
        ix = Index(c.n, c.cfg.dim, c.cfg.vocab, 100, dtype=dtype, rescore_r=r,
                   max_batch=max(sizes), n_workspaces=2)
        ix.load_corpus(c.emb, c.ids, c.term_off, c.terms)
        for n in sizes:
            qb = pool.subset(range(2048 - n, 2048))
            choice = ix.autotune(qb.emb, qb, 100)
            print(f"[tune] {dtype} Q={n}: (query_blocks, waves, groups, strategy) = {choice}",
                  flush=True)
        with tempfile.TemporaryDirectory() as d:
            path = os.path.join(d, "t.jsonl")
            ix.tuning_save(path)
            lines += open(path).read().splitlines()
        ix.close()
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"[tune] {len(lines)} entries -> {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
