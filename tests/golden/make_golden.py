"""Writes the hand-derived worked examples in this folder.

Nothing here calls the oracle or the HIP library: each expected value is a
closed form derived on paper from the method's definitions, and the
derivation is stored next to the numbers.
"""
import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def tonemap_paper_inverse():
    # Section 3.4 listing: forward res /= (1 + luma(res) * lumaMultiplier),
    # "removal" specular * (1 + luma(specular)) * reinhardToneMappingWeight.
    # For a grey pixel (luma = c) with multiplier = weight = 1:
    #   c' = c / (1 + c),   c'' = c' (1 + c') = c (1 + 2c) / (1 + c)^2.
    cases = [{"L": L, "ratio": (1 + 2 * L) / (1 + L) ** 2} for L in (0.1, 0.5, 1.0, 2.0, 10.0)]
    return {
        "source": "Section 3.4 (Reinhard tone mapping listing)",
        "derivation": "grey c, k = w = 1: paper_inverse(T(c)) / c = (1 + 2c) / (1 + c)^2; 0.75 at c = 1",
        "cases": cases,
    }


def atrous_luma_example():
    # One-row image (H = 1), step 1, flat depth and equal normals, so depth
    # and normal weights are 1 and only taps (a, 0) lie in the image: B3
    # weights 1/16, 1/4, 3/8, 1/4, 1/16 along x.  The luminance weight is
    # exp(-|dL| / (sigma_l sqrt(g))) with g the 3x3 Gaussian (1/4, 1/2, 1/4)
    # of the variance (one row: 0.25 v[x-1] + 0.5 v[x] + 0.25 v[x+1]).
    # Neighbours at dL = 8 ln 2 with sigma_l sqrt(g) = 8 weigh exactly 1/2.
    v = 1.0 + 8.0 * math.log(2.0)
    cases = []
    # all four neighbours at +8 ln 2, g = 4, sigma_l = 4
    for var in ([4.0] * 5, [1.0, 2.0, 6.0, 2.0, 1.0]):
        cases.append({
            "grey": [v, v, 1.0, v, v], "var": var, "sigma_l": 4.0, "x": 2,
            "expect": (3 / 8 * 1.0 + 0.5 * (5 / 8) * v) / (3 / 8 + 0.5 * 5 / 8),
            "why": "g = 4 (prefiltered), w = 1/2 on all four neighbours",
        })
    cases.append({
        "grey": [v, v, 1.0, v, v], "var": [16.0] * 5, "sigma_l": 2.0, "x": 2,
        "expect": (3 / 8 * 1.0 + 0.5 * (5 / 8) * v) / (3 / 8 + 0.5 * 5 / 8),
        "why": "sigma_l sqrt(g) = 2 * 4 = 8",
    })
    # outer neighbours equal to p (w = 1), inner ones at +8 ln 2 (w = 1/2)
    cases.append({
        "grey": [1.0, v, 1.0, v, 1.0], "var": [4.0] * 5, "sigma_l": 4.0, "x": 2,
        "expect": (3 / 8 + 2 / 16 + 0.5 * 2 / 4 * v) / (3 / 8 + 2 / 16 + 0.5 * 2 / 4),
        "why": "w = 1 at a = +-2, w = 1/2 at a = +-1",
    })
    return {
        "source": "Section 2 (edge-avoiding a-trous with a variance-guided luminance weight)",
        "derivation": "see make_golden.py",
        "cases": cases,
    }


def main():
    for name, fn in (("tonemap_paper_inverse.json", tonemap_paper_inverse),
                     ("atrous_luma_example.json", atrous_luma_example)):
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(fn(), f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
