"""Autotune the fused signed-distance tiles for the named workloads and write
the table the benchmark ships with (one line per shape, see mppi_tune_get).

    python -m paper_2605_29663_amd.tune --out paper_2605_29663_amd/tiles_gfx950.txt
"""
from __future__ import annotations

import argparse


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--configs", default="c1,c2,c3")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    import paper_2605_29663_amd as pkg
    from paper_2605_29663_amd import scenes
    lines = []
    for name in args.configs.split(","):
        prm, sc = scenes.config(name)
        ctx = pkg.Context(0)
        kind = prm["footprint_kind"]
        ctx.set_footprint(kind, sc["polygon"] if kind == 0 else sc["rects"])
        ctx.set_points(sc["ox"], sc["oy"], sc.get("ovx"), sc.get("ovy"))
        blk, nc = ctx.mppi_autotune(prm, reps=args.reps)
        print(f"{name}: block {blk}, chunks {nc}", flush=True)
        lines += ctx.mppi_tune_get().splitlines()
        ctx.close()
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
