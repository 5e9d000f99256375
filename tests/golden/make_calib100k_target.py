"""Write calib100k_target_incidence.txt: the relaxed daily incidence of the 100,000-agent
calibration population over 180 days at parameters other than the reference ones,
computed by the FP64 oracle alone (no GPU).  The full-size adjoint test uses it as
the target curve c* of the loss sum_t (c(t) - c*(t))^2 / T.

    python tests/golden/make_calib100k_target.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.soft import SoftModel  # noqa: E402
from synthpop import workload  # noqa: E402

T = 180
R_TARGET = 4.6
S_TARGET = np.linspace(0.5, 1.2, 9)


def main():
    p, pop = workload(4, n_steps=T)
    c, _, _ = SoftModel(pop, p, R=np.array([R_TARGET]), S=S_TARGET[None, :]).run(T, tangents=False)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "calib100k_target_incidence.txt")
    with open(out, "w") as f:
        f.write("# relaxed daily incidence, calib-100k population (workload 4), 180 days, FP64 oracle\n")
        f.write(f"# R = {R_TARGET}, S = linspace(0.5, 1.2, 9); written by make_calib100k_target.py\n")
        for v in c[0]:
            f.write(f"{v:.17g}\n")


if __name__ == "__main__":
    main()
