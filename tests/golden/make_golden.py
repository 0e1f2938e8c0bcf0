"""Write the oracle's moments for the full-size workloads into tests/golden/ (CPU only).

Every stored value comes from the CPU oracle (oracle/), never from the HIP path:

  config2_oracle.txt   3D 64^3 spin hopping, M=1024, R=32 phase vectors (seed 1002, instance 0)
  config4_oracle.txt   2D 2048^2 Anderson, all M=4096 moments, R=64 +-1 (seed 1004, instance 0)
                       (about 80 minutes of oracle time on 8 threads)
  config3_h<h>_oracle.txt  instances h of the 256-cube batch, M=512, R=16 phase (seed 1003,
                       instance h): 0..3 (the first four), and CONFIG3_EXTRA, which adds every
                       L=48 cube (8, 78, 209) and cubes of L = 47, 46, 45, 44, 40, 21, 17

The scale (a, b) is the oracle's Gershgorin bound with margin 0.01; it is stored (as hex) with
the moments so the GPU tests use exactly the same operator.

Usage: python tests/golden/make_golden.py [config2] [config3] [config4]
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1105_5481_amd import workloads as wl  # noqa: E402


# config-3 instances beyond the first four: indices of the L = 48 cubes and of a spread of sizes
CONFIG3_EXTRA = (8, 78, 209, 12, 38, 19, 4, 7, 11, 29)


def bounds(lat):
    lo, hi = oracle.gershgorin_lattice(lat.dim, lat.L[:lat.dim], lat.t, lat.hop, lat.onsite, lat.spinor)
    return oracle.scale_from_bounds(lo, hi, 0.01)


def write(path, header, mu):
    with open(path, "w") as f:
        for k, v in header.items():
            f.write(f"# {k}: {v}\n")
        for x in mu:
            f.write(f"{float(x).hex()}\n")


def run(lat, M, R, vec, seed, instance):
    a, b = bounds(lat)
    t0 = time.time()
    mu = oracle.moments_lattice(lat.dim, lat.L[:lat.dim], lat.t, a, b, M, R, vec_kind=vec, seed=seed,
                                instance=instance, hop=lat.hop, onsite=lat.onsite, spinor=lat.spinor)
    return a, b, mu, time.time() - t0


def main(which):
    oracle.build()
    if "config2" in which:
        cfg = wl.config2()
        a, b, mu, dt = run(cfg["lattice"], cfg["M"], cfg["R"], cfg["vec"], cfg["seed"], 0)
        write(os.path.join(HERE, "config2_oracle.txt"),
              {"workload": cfg["name"], "M": cfg["M"], "R": cfg["R"], "vec": cfg["vec"], "seed": cfg["seed"],
               "instance": 0, "a": a.hex(), "b": b.hex(), "oracle_seconds": f"{dt:.1f}"}, mu)
        print("config2", dt, flush=True)
    if "config4" in which:
        cfg = wl.config4()
        a, b, mu, dt = run(cfg["lattice"], cfg["M"], cfg["R"], cfg["vec"], cfg["seed"], 0)
        write(os.path.join(HERE, "config4_oracle.txt"),
              {"workload": cfg["name"], "M": cfg["M"], "R": cfg["R"], "vec": cfg["vec"],
               "seed": cfg["seed"], "instance": 0, "a": a.hex(), "b": b.hex(), "oracle_seconds": f"{dt:.1f}"}, mu)
        print("config4", dt, flush=True)
    if "config3" in which:
        cfg = wl.config3()
        for h in list(range(4)) + list(CONFIG3_EXTRA):
            lat = cfg["lattices"][h]
            a, b, mu, dt = run(lat, cfg["M"], cfg["R"], cfg["vec"], cfg["seed"], h)
            write(os.path.join(HERE, f"config3_h{h}_oracle.txt"),
                  {"workload": cfg["name"] + f" instance {h}", "L": lat.L[0], "M": cfg["M"], "R": cfg["R"],
                   "vec": cfg["vec"], "seed": cfg["seed"], "instance": h, "a": a.hex(), "b": b.hex(),
                   "oracle_seconds": f"{dt:.1f}"}, mu)
            print("config3", h, lat.L[0], dt, flush=True)


def load(path):
    """(header dict, moments) from a golden file."""
    hdr, mu = {}, []
    for line in open(path):
        if line.startswith("#"):
            k, v = line[1:].split(":", 1)
            hdr[k.strip()] = v.strip()
        elif line.strip():
            mu.append(float.fromhex(line.strip()))
    return hdr, mu


if __name__ == "__main__":
    main(sys.argv[1:] or ["config2", "config3", "config4"])
