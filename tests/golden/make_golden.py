"""Writes the stored expected inputs under tests/golden/ using only the oracle.

cfg1_target_128.npy: the 1,000-Gaussian single-view workload's target image,
the seed-1 Gaussian set rendered by the FP64 oracle through the 128x128,
60-degree axis camera at distance 3, stored as float32 RGBA [4][128][128].

Run:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth   # noqa: E402


def main():
    P1 = synth.random_gaussians(1000, seed=synth.SEED_TARGET_SET)
    cam = synth.axis_camera(128, 128)
    r = oracle.render(P1, cam)
    img = r.rgba.reshape(4, 128, 128).astype(np.float32)
    np.save(os.path.join(HERE, "cfg1_target_128.npy"), img)
    print("wrote cfg1_target_128.npy", img.shape, float(img[3].mean()))


if __name__ == "__main__":
    main()
