"""Write hartmann_c2_oracle.json: the FP64 oracle's steady Hartmann profile.

Runs only the CPU oracle (oracle/) on the x-invariant 1 x 256 column of the
512 x 256 channel (G = 1e-6, Ha = 10, tau_f = 0.6, tau_m = 0.55, walls in y,
insulating walls imposing b = (0, B0)) from rest until the largest change of
u over 10^4 steps is below 1e-12, and stores u_x(y), b_x(y), b_y(y).
Usage: python tests/golden/make_hartmann_c2.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2602_14667_amd import inputs  # noqa: E402


def main():
    h = inputs.hartmann_c2()
    o = oracle.Oracle(1, h.ny, h.tau_f, h.tau_m, walls=True, force=(h.G, 0.0),
                      b_wall=(0.0, h.B0))
    u, b = h.initial_fields()
    o.init(u[:, :, :1], b[:, :, :1])
    _, prev, _ = o.moments()
    chunk = 10000
    while True:
        o.step(chunk)
        _, v, c = o.moments()
        change = float(np.max(np.abs(v - prev)))
        prev = v
        if change < 1e-12:
            break
    rho, v, c = o.moments()
    out = {
        "what": "FP64 oracle steady state of the 512x256 Hartmann channel "
                "(x-invariant column), started from rest",
        "ny": h.ny, "tau_f": h.tau_f, "tau_m": h.tau_m, "G": h.G, "Ha": h.Ha,
        "B0": h.B0, "steps": o.step_count,
        "max_change_last_10k_steps": change,
        "ux": v[0, :, 0].tolist(), "bx": c[0, :, 0].tolist(),
        "by": c[1, :, 0].tolist(), "rho": rho[:, 0].tolist(),
    }
    with open(os.path.join(HERE, "hartmann_c2_oracle.json"), "w") as fh:
        json.dump(out, fh)
    print(o.step_count, change)


if __name__ == "__main__":
    main()
