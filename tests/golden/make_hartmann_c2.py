"""Write hartmann_c2_oracle.json: FP64 oracle profiles of the Hartmann channel.

Runs only the CPU oracle (oracle/) on the x-invariant 1 x 256 column of the
512 x 256 channel (G = 1e-6, Ha = 10, tau_f = 0.6, tau_m = 0.55, walls in y,
insulating walls imposing b = (0, B0)), started from the closed-form profile,
for 400,000 steps (1.5 e-foldings of the slowest mode), twice: in plain FP64,
and with the state rounded after every step to what FP32 storage keeps (the
storage-precision model, f - w and g to the nearest FP32 value).  Stores
u_x(y), b_x(y), b_y(y) and rho(y) of both runs.
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

STEPS = 400_000


def closed_form_fields(h):
    ue, be = h.profile(np.arange(h.ny))
    u = np.zeros((2, h.ny, 1))
    b = np.zeros((2, h.ny, 1))
    u[0, :, 0] = ue
    b[0, :, 0] = be
    b[1] = h.B0
    return u, b


def run(h, rounded):
    o = oracle.Oracle(1, h.ny, h.tau_f, h.tau_m, walls=True, force=(h.G, 0.0),
                      b_wall=(0.0, h.B0))
    u, b = closed_form_fields(h)
    o.init(u, b)
    if rounded:
        o.round_state_f32()
        o.step_rounded_f32(STEPS)
    else:
        o.step(STEPS)
    rho, v, c = o.moments()
    return {"ux": v[0, :, 0].tolist(), "bx": c[0, :, 0].tolist(),
            "by": c[1, :, 0].tolist(), "rho": rho[:, 0].tolist()}


def main():
    h = inputs.hartmann_c2()
    out = {
        "what": "FP64 oracle on the x-invariant column of the 512x256 Hartmann "
                "channel, started from the closed-form profile; 'fp64' plain, "
                "'fp32_storage' with the state rounded to FP32 storage after "
                "every step",
        "ny": h.ny, "tau_f": h.tau_f, "tau_m": h.tau_m, "G": h.G, "Ha": h.Ha,
        "B0": h.B0, "steps": STEPS, "start": "closed form",
        "fp64": run(h, False), "fp32_storage": run(h, True),
    }
    with open(os.path.join(HERE, "hartmann_c2_oracle.json"), "w") as fh:
        json.dump(out, fh)
    a, r = out["fp64"], out["fp32_storage"]
    for k in ("ux", "bx", "by"):
        x, y = np.array(a[k]), np.array(r[k])
        print(k, np.linalg.norm(y - x) / np.linalg.norm(x))


if __name__ == "__main__":
    main()
