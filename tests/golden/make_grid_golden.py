"""Write the reference amplitude of the 6x6, depth-8 fSim grid circuit.

Calls only the oracle (O2, complex128 tensor-network sweeps) and the seeded
workload generator.  Two independent sweep orders (column-major and
row-major) are run; both values are stored and must agree to 1e-12
relative.  Needs about 30 GB of host memory and several minutes per order.

    python tests/golden/make_grid_golden.py [rows cols depth]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import tcgen  # noqa: E402
from oracle import tn  # noqa: E402


def main():
    rows, cols, depth = (int(a) for a in sys.argv[1:4]) if len(sys.argv) > 3 else (6, 6, 8)
    circ, params, _ = tcgen.workload_grid_amplitude(rows, cols, depth)
    out = {"_about": "Reference amplitude <0^n|U|0^n> of the seeded fSim grid "
                     "workload (structure seed 3, angle seed 4), computed by "
                     "oracle/tn.py in complex128 with two sweep orders.",
           "rows": rows, "cols": cols, "depth": depth,
           "struct_seed": 3, "param_seed": 4, "values": {}}
    for order in ("col2", "row2"):
        t0 = time.time()
        ts = sorted(tn.amplitude_network(circ, params), key=tn._sort_key(order))
        peak = tn.peak_log2(ts)
        print(f"order {order}: peak 2^{peak} elements", flush=True)
        a = tn._fold(ts, 1 << 30)
        dt = time.time() - t0
        print(f"order {order}: {a!r} in {dt:.1f} s", flush=True)
        out["values"][order] = {"re": a.real, "im": a.imag, "peak_log2": peak,
                                "seconds": round(dt, 1)}
    v = [complex(x["re"], x["im"]) for x in out["values"].values()]
    rel = abs(v[0] - v[1]) / abs(v[0])
    out["order_agreement_rel"] = rel
    print("relative difference between orders:", rel, flush=True)
    path = os.path.join(HERE, f"grid{rows}x{cols}_d{depth}_amplitude.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
