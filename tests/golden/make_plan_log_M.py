"""Writes plan_log_M.txt: the oracle's rejection constants (Nelder-Mead from
the zero-mean Dirichlet kernel plus further starts, oracle/plan.py) of the
points the GPU search is checked on.  Calls only the oracle.

    python tests/golden/make_plan_log_M.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import plan as OP  # noqa: E402

POINTS = [  # K, E0, beta', C3/C2, proposal (1 Sigma, 0 uniform)
    (2, 1.0, 3.0, 5.0, 1), (2, 1.0, 3.0, -5.0, 0), (3, 1.0, 5.0, 4.0, 1), (7, 0.5, 12.0, 15.0, 1),
    (8, 1.0, 40.0, 20.0, 1), (8, 1.0, 40.0, 20.0, 0), (16, 1.0, 40.0, 60.0, 1), (16, 1.0, 40.0, 30.0, 0),
    (16, 2.0, 60.0, 100.0, 1), (32, 1.0, 40.0, 75.0, 1), (32, 1.0, 20.0, 300.0, 1), (32, 1.0, 40.0, -75.0, 1),
    (48, 1.0, 30.0, 120.0, 1), (64, 1.0, 40.0, 150.0, 1),
]


def main():
    lines = ["# K E0 beta' C3/C2 proposal log_M   (oracle/plan.py log_M, n_random=2)"]
    for K, E0, bp, c, prop in POINTS:
        a = OP.alpha_star(K, bp) if prop == 1 else 1.0
        lm, _ = OP.log_M(K, E0, bp, c, prop, a, n_random=2)
        lines.append(f"{K} {E0!r} {bp!r} {c!r} {prop} {lm!r}")
        print(lines[-1], flush=True)
    with open(os.path.join(HERE, "plan_log_M.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
