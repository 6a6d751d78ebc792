"""Write tests/golden/tables_oracle.txt: the oracle's errors for the paper's Table 1 and
Table 2 runs (all three schemes), which the GPU tests compare against.  Calls only the oracle.

    python tests/golden/make_tables_oracle.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O          # noqa: E402
from tests import paper_tables as PT    # noqa: E402


def main():
    lines = ["# Oracle errors of the paper's Table 1 (wave) and Table 2 (shock) runs, written by",
             "# tests/golden/make_tables_oracle.py from the FP64 oracle alone.",
             "# columns: kind  h  tau  method  error"]
    for kind, name in (("wave", "table1_dustywave.txt"), ("shock", "table2_dustyshock.txt")):
        for h, tau, _ in PT.printed(name):
            for m in ("MK", "ISPH", "IDIC"):
                prob = (PT.wave_problem if kind == "wave" else PT.shock_problem)(h, tau, m)
                x, u = PT.run_oracle(O, prob)
                err = (PT.wave_error if kind == "wave" else PT.shock_error)(prob, x, u)
                lines.append(f"{kind} {h:g} {tau:g} {m} {err:.12e}")
                print(lines[-1], flush=True)
    with open(os.path.join(HERE, "tables_oracle.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
