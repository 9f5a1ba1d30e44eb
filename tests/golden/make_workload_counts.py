"""Write tests/golden/workload_counts.json: the algorithmic work of one frame of each benchmark
workload, counted by the FP64 oracle (nothing here touches the GPU library).

Per workload: pixels, tiles, P (tile-Gaussian pairs), F (list entries the tiles must fetch),
E (pair evaluations until each pixel stops), Eb (pairs the backward revisits: positions before
each pixel's last contributor) and K (blended pairs). The roofline of the blend kernels multiplies
these by the per-pair operation counts stated in the design notes.

Run:  python tests/golden/make_workload_counts.py [C2 C3 ...]
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gsinputs  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "workload_counts.json")


def counts(name: str) -> dict:
    s = gsinputs.make_scene(name)
    f = oracle.render(s)
    c = oracle.work_counts(f, f["ranges"])
    gx, gy = oracle.grid(s["width"], s["height"])
    c.update({"width": s["width"], "height": s["height"], "gaussians": int(len(s["radii"])),
              "pixels": s["width"] * s["height"], "tiles": gx * gy,
              "seed": gsinputs.CONFIGS[name].seed})
    return c


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data["_source"] = ("oracle/ (FP64) on the seeded scenes of gsinputs; written by "
                       "tests/golden/make_workload_counts.py")
    for n in names:
        data[n] = counts(n)
        print(n, data[n], flush=True)
    with open(OUT, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or ["C2", "C3"])
