"""Write the exact wet-bed dam-break (Stoker) constants used by the oracle pins.

The solution of the 1D shallow-water Riemann problem with still water of
depth h_L left of the dam and h_R right of it (flat frictionless bed) is a
left rarefaction and a right shock around a middle state (h_m, u_m) fixed by

    u_m = 2 (sqrt(g h_L) - sqrt(g h_m))                       (rarefaction)
    u_m = (h_m - h_R) sqrt(g (h_m + h_R) / (2 h_m h_R))         (shock)

with shock speed S = h_m u_m / (h_m - h_R).  Solved here to 30 digits with
mpmath (textbook closed form, independent of the oracle).
Run:  python tests/golden/make_stoker.py
"""
import json
import os

import mpmath as mp

mp.mp.dps = 30


def solve(hL, hR, g):
    cL = mp.sqrt(g * hL)

    def f(hm):
        return 2 * (cL - mp.sqrt(g * hm)) - (hm - hR) * mp.sqrt(g * (hm + hR) / (2 * hm * hR))

    hm = mp.findroot(f, (hR * 1.0001, hL * 0.9999), solver="anderson")
    um = 2 * (cL - mp.sqrt(g * hm))
    S = hm * um / (hm - hR)
    return dict(h_L=float(hL), h_R=float(hR), g=float(g), h_m=float(hm), u_m=float(um),
                shock_speed=float(S), head_speed=float(-cL),
                tail_speed=float(um - mp.sqrt(g * hm)))


if __name__ == "__main__":
    out = solve(mp.mpf("1.0"), mp.mpf("0.5"), mp.mpf("9.81"))
    out["source"] = ("exact Riemann solution of the SWE (textbook closed form); "
                     "dam-break depths 1.0 m / 0.5 m as in the dam-break workload")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stoker_dambreak.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))
