"""Write n2p_oracle_design.json: the FP64 oracle's own run of the N2P lens
design loop (Sec. VI) at three lens thicknesses, for the GPU design loop to be
compared with.  Calls only ``oracle`` (and the input generators).

    python tests/golden/make_n2p_oracle_design.py      # a few minutes on 8 cores
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

import oracle  # noqa: E402
from oracle import n2p  # noqa: E402

SEARCH = {"beta": (0.2, 2.5), "gamma": (0.5, 8.0), "grid": 33, "window": 3, "levels": 12,
          "tol": 1e-5}


def main():
    oracle.build()
    out = {"source": "FP64 oracle (oracle/n2p.py) running the successive-refinement search of "
                     "Sec. VI on the N2P lens of Eq. (27), scored by Eqs. (28)-(29); R = 1, "
                     "F = 2R, N = 10 rays at y_i = 0.995 R i / N, dL0 = 1e-4 R",
           "search": SEARCH, "designs": []}
    for L in (0.2, 0.3, 1.0):
        t0 = time.time()
        b, g, e, lev = n2p.design(L, **SEARCH)
        out["designs"].append({"L": L, "beta": b, "gamma": g, "rmse_lsa": e,
                               "levels": [list(x) for x in lev]})
        print(f"L={L}: beta={b:.6f} gamma={g:.6f} rmse={e:.4e} ({time.time() - t0:.0f} s)",
              flush=True)
    with open(os.path.join(HERE, "n2p_oracle_design.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
