"""Writes the stored expected values under tests/golden/ that are not worked by hand.

It calls only the oracle package and the input generator, never the HIP
library.  Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1306_1373_amd.synth import digest, synth_image  # noqa: E402

# (W, H, seed, sigma) of the images the tests regenerate
SYNTH_CASES = [(512, 512, s, 5.0) for s in range(4)] + [
    (1024, 814, 0, 5.0), (200, 200, 1, 5.0), (7, 9, 2, 3.0), (1, 1, 3, 0.0), (544, 512, 4, 10.0)]


def main():
    digests = []
    for W, H, seed, sigma in SYNTH_CASES:
        digests.append({"W": W, "H": H, "seed": seed, "sigma": sigma,
                        "sha256": digest(synth_image(W, H, seed, sigma))})
    with open(os.path.join(HERE, "synth_digests.json"), "w") as f:
        json.dump({"generator": "paper_1306_1373_amd.synth.synth_image", "cases": digests}, f,
                  indent=1)

    # oracle regression record: SSE and PSNR of the recipe codec on the 512 x 512 images
    rec = []
    for seed in range(4):
        img = synth_image(512, 512, seed, 5.0)
        for qs in (2, 4, 8, 16):
            _, s = oracle.cordic_codec(img, qs)
            rec.append({"seed": seed, "qs": qs, "sse": s,
                        "psnr": oracle.psnr_from_sse(s, 512, 512)})
    with open(os.path.join(HERE, "oracle_codec_512.json"), "w") as f:
        json.dump({"written_by": "tests/golden/make_golden.py (oracle only)",
                   "workload": "512x512 synthetic, sigma 5", "cases": rec}, f, indent=1)


if __name__ == "__main__":
    main()
