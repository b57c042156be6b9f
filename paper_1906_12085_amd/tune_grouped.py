"""Autotune the tile parameters of grouped batches (rsvd_batch_grouped_tune)
on the 512-instance batched workload and write them to a cache file, by
default tune_grouped_gfx950.json beside this module, which
load_tune_cache() reads for rsvd_batch_grouped_create.

    python -m paper_1906_12085_amd.tune_grouped [OUT.json]

Run from the repository root (the input generator `synth` is imported from
there) on an MI355X.  The tuner times grouped launches of each (n, l)
bucket's instances alone, so the entries are measured, not modelled.
"""
from __future__ import annotations

import json
import sys
import time


def main(argv=None) -> int:
    argv = sys.argv[1:] if argv is None else argv
    import torch

    import synth
    from paper_1906_12085_amd import TUNE_CACHE, Batch

    out = argv[0] if argv else TUNE_CACHE
    c = synth.CONFIG4
    dev = torch.device("cuda", 0)
    shapes = synth.batch_shapes(c)
    probs = synth.batch_problems(torch, dev, c)
    torch.cuda.synchronize()
    mmax = max(s[0] for s in shapes)
    nmax = max(s[1] for s in shapes)
    lmax = max(min(s[3] + c["p"], s[1]) for s in shapes)
    b = Batch(1, mmax, nmax, lmax, torch.float32, seed=c["seed"])
    t0 = time.perf_counter()
    entries = b.tune_grouped(probs)
    secs = time.perf_counter() - t0
    b.close()
    data = {
        "arch": "gfx950",
        "device": torch.cuda.get_device_name(0),
        "workload": (f"{c['count']} fp32 instances, m uniform in [{c['m_lo']}, {c['m_hi']}], "
                     f"n in {list(c['n_choices'])}, k = min({c['k_max']}, n/4), p = {c['p']}, "
                     f"q = {c['q']}"),
        "tuning_seconds": round(secs, 1),
        "entries": [dict(n=n, l=l, panel_rows=pr, split_rows=sr) for n, l, pr, sr in entries],
    }
    with open(out, "w") as f:
        json.dump(data, f, indent=1)
        f.write("\n")
    print(json.dumps(data))
    return 0


if __name__ == "__main__":
    sys.exit(main())
