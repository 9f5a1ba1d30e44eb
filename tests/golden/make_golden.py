"""Write the closed-form fixtures of tests/golden/ with exact rational arithmetic.

Nothing here calls the oracle or the GPU library: the values follow from Eq. (volume-render) and
the per-pixel loop of Alg. 1 (alpha-skip, early termination), evaluated by hand in exact
arithmetic (``fractions.Fraction``) for stacks of Gaussians centred on the pixel, where the
exponent is 0 and alpha equals the opacity exactly.

Run:  python tests/golden/make_golden.py
"""
import json
import os
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
T_STOP = Fraction(float(np.float32(1e-4)))


def composite(alphas, colors, bg):
    """Front-to-back: T' = T(1 - a); stop (without blending) once T' < 1e-4."""
    T = Fraction(1)
    acc = [Fraction(0)] * 3
    Ts, last = [], 0
    for k, (a, c) in enumerate(zip(alphas, colors)):
        Tn = T * (1 - a)
        if Tn < T_STOP:
            break
        for ch in range(3):
            acc[ch] += a * T * c[ch]
        T = Tn
        Ts.append(T)
        last = k + 1
    image = [acc[ch] + T * bg[ch] for ch in range(3)]
    return image, T, last, Ts


def main():
    # Six identical Gaussians at the pixel, opacity fp32(0.8): T = 0.2^k; the 6th would give
    # T' ~ 6.4e-5 < 1e-4, so it stops there with five blended.
    a = Fraction(float(np.float32(0.8)))
    col = [Fraction(float(np.float32(v))) for v in (1.0, 0.5, 0.25)]
    image, T, last, Ts = composite([a] * 6, [col] * 6, [Fraction(0)] * 3)
    five = {
        "source": "Eq. (volume-render) + early termination of Alg. 1 (T' < 1e-4 tested before "
                  "blending); six identical Gaussians centred on pixel (8, 8), opacity fp32(0.8), "
                  "colour (1, 0.5, 0.25), depths 1..6, black background",
        "pixel": [8, 8], "n": 6, "opacity": float(np.float32(0.8)),
        "T_after_each": [float(t) for t in Ts],
        "last_contrib": last, "final_T": float(T), "image": [float(v) for v in image],
    }
    with open(os.path.join(HERE, "five_stack.json"), "w") as f:
        json.dump(five, f, indent=1)
        f.write("\n")

    # Two Gaussians at the pixel, front one first: C = a1 c1 + (1 - a1) a2 c2 + (1-a1)(1-a2) bg
    o1, o2 = Fraction(float(np.float32(0.6))), Fraction(float(np.float32(0.3)))
    c1 = [Fraction(float(np.float32(v))) for v in (0.9, 0.1, 0.2)]
    c2 = [Fraction(float(np.float32(v))) for v in (0.2, 0.7, 0.4)]
    bg = [Fraction(float(np.float32(v))) for v in (0.25, 0.5, 0.75)]
    img12, T12, last12, _ = composite([o1, o2], [c1, c2], bg)
    img21, T21, last21, _ = composite([o2, o1], [c2, c1], bg)
    two = {
        "source": "Eq. (volume-render): C = a1 c1 + (1 - a1) a2 c2 + T bg for two Gaussians "
                  "centred on pixel (3, 5) of a 16x16 image; depths (1, 2) then swapped",
        "pixel": [3, 5], "opacity": [float(o1), float(o2)],
        "colors": [[float(v) for v in c1], [float(v) for v in c2]],
        "bg": [float(v) for v in bg],
        "front_first": {"image": [float(v) for v in img12], "final_T": float(T12), "last_contrib": last12},
        "swapped": {"image": [float(v) for v in img21], "final_T": float(T21), "last_contrib": last21},
    }
    with open(os.path.join(HERE, "two_stack.json"), "w") as f:
        json.dump(two, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
