"""Writes tests/golden/oracle_values.json from the oracle alone (closed form + FP64 MPS).

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import closed_form, mps  # noqa: E402
from paper_2601_03832_amd import inputs  # noqa: E402


def main():
    out = {"p_marked_final": {}, "c1_schmidt": {}, "c1_bond_dims": None}
    for w in (inputs.config_c1(), inputs.config_c2(), inputs.config_c3(), inputs.config_c5(count=1)):
        i = w.instances[0]
        out["p_marked_final"][w.name] = {"n": i.n, "M": i.M, "k": i.k,
                                         "p": closed_form.p_marked(i.n, i.M, i.k)}
    c1 = inputs.config_c1().instances[0]
    m = mps.run(c1.n, c1.marked, c1.k, c1.chi_cap)
    for cut in range(1, c1.n):
        out["c1_schmidt"][str(cut)] = [float(v) for v in m.schmidt_values(cut)]
    out["c1_bond_dims"] = m.bond_dims()
    out["c1_marked"] = [int(x) for x in c1.marked]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print("wrote", path)


if __name__ == "__main__":
    main()
