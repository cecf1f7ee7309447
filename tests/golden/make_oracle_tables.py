"""Write tests/golden/oracle_soe_tables.json from the oracle's own table builder.

Calls only ``oracle.soe_table`` (Sections 2-3 of the paper: the Section 3.4
hyperbolic contour, the midpoint rule (2.7)-(2.9) and balanced truncation,
Section 2.4).  Run from the repository root:

    python tests/golden/make_oracle_tables.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import soe_table  # noqa: E402


def main():
    out = {"source": "oracle.soe_table: Section 3.4 contour, n=%d nodes, midpoint rule, "
                     "balanced truncation (Section 2.4), E_n on the (3.1) grid" % soe_table.CONTOUR_N,
           "tables": {}}
    for m in range(1, 8):
        t = soe_table.gaussian_table(m)
        out["tables"][str(m)] = {
            "n_modes": m,
            "tau0_re": [float(v.real) for v in t["tau0"]],
            "tau0_im": [float(v.imag) for v in t["tau0"]],
            "omega_re": [float(v.real) for v in t["omega"]],
            "omega_im": [float(v.imag) for v in t["omega"]],
            "E": t["E"], "Eprime": t["Eprime"], "max_imag": t["max_imag"],
            "sum_abs_omega": t["sum_abs_omega"],
        }
        print(m, "E=%.3e E'=%.3e sum|w|=%.3g" % (t["E"], t["Eprime"], t["sum_abs_omega"]), flush=True)
    with open(os.path.join(HERE, "oracle_soe_tables.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
