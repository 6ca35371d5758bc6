"""Writes the golden ECC files of this directory.  Calls only the oracle.

Each file holds one ECC (int64 per bin, one per line) for a seeded synthetic
input; its header names the input, the filtration and the bin count.  Run from
the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2203_09087_amd import synth  # noqa: E402

CASES = {
    # name: (description, image factory, nbins, value range)
    "uniform_256x256_u8_seed1": ("256x256 uint8 i.i.d. uniform gray levels, seed 1",
                                 lambda: synth.uniform_u8((256, 256), seed=1), 256, None),
    "smoothed_64cubed_u8_seed7": ("64^3 uint8 white noise smoothed (sigma 2), 256 levels, seed 7",
                                  lambda: synth.smoothed_noise_u8((64, 64, 64), 2.0, seed=7), 256, None),
}


def main():
    oracle.build(force=False)
    for name, (desc, make, nbins, rng) in CASES.items():
        img = make()
        for cons in ("vertex", "top"):
            curve = oracle.ecc(img, nbins, cons, value_range=rng, threads=8)
            path = os.path.join(HERE, f"{name}_{cons}.txt")
            with open(path, "w") as f:
                f.write(f"# ECC of {desc}; {cons} filtration; {nbins} bins; written by make_golden.py (oracle)\n")
                f.write("\n".join(str(int(v)) for v in curve) + "\n")
            print("wrote", path)


if __name__ == "__main__":
    main()
