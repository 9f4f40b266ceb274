"""Write the reference amplitude of a seeded fSim grid circuit.

Calls only the oracle (complex128) and the seeded workload generator.  Two
independent methods are run; both values are stored and must agree to 1e-12
relative.  Methods: the tensor-network sweeps of oracle/tn.py in one of the
orders "col", "row", "col2", "row2", "time", or "statevector" (the gate-by-
gate state vector of oracle/statevector.py).  The default pair, column- and
row-major sweeps, suits the 6x6 depth-8 grid (about 30 GB of host memory
and several minutes per order); deeper, narrower grids whose sweeps peak
too high take "time statevector" (the 4x6 depth-12 grid: about a minute
each).

    python tests/golden/make_grid_golden.py [rows cols depth [method method]]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import tcgen  # noqa: E402
from oracle import statevector as sv  # noqa: E402
from oracle import tn  # noqa: E402


def main():
    rows, cols, depth = (int(a) for a in sys.argv[1:4]) if len(sys.argv) > 3 else (6, 6, 8)
    methods = sys.argv[4:6] if len(sys.argv) > 5 else ["col2", "row2"]
    circ, params, _ = tcgen.workload_grid_amplitude(rows, cols, depth)
    out = {"_about": "Reference amplitude <0^n|U|0^n> of the seeded fSim grid "
                     "workload (structure seed 3, angle seed 4), computed in "
                     "complex128 by two methods of the oracle: " + ", ".join(
                         "state vector" if m == "statevector" else f"tensor-network sweep ({m} order)"
                         for m in methods) + ".",
           "rows": rows, "cols": cols, "depth": depth,
           "struct_seed": 3, "param_seed": 4, "values": {}}
    for m in methods:
        t0 = time.time()
        if m == "statevector":
            peak = circ.n_qubits
            a = complex(sv.amplitude(circ, params))
        else:
            ts = sorted(tn.amplitude_network(circ, params), key=tn._sort_key(m))
            peak = tn.peak_log2(ts)
            print(f"order {m}: peak 2^{peak} elements", flush=True)
            a = tn._fold(ts, 1 << 30)
        dt = time.time() - t0
        print(f"{m}: {a!r} in {dt:.1f} s", flush=True)
        out["values"][m] = {"re": a.real, "im": a.imag, "peak_log2": peak,
                            "seconds": round(dt, 1)}
    v = [complex(x["re"], x["im"]) for x in out["values"].values()]
    rel = abs(v[0] - v[1]) / abs(v[0])
    out["order_agreement_rel"] = rel
    print("relative difference between methods:", rel, flush=True)
    if rel > 1e-12:
        raise SystemExit("the two methods disagree")
    path = os.path.join(HERE, f"grid{rows}x{cols}_d{depth}_amplitude.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
