#!/usr/bin/env python3
"""Writes stability_counts.txt beside this file: for every named parity
workload (tests/parity_workloads.py), how many of its fitness cases the
oracle's stability classifier marks stable, envelope, non-finite stable or
unchecked, and how many individuals fall in each fitness class of the parity
contract (tests/_parity.py).  Runs the CPU oracle only.

    python tests/golden/write_stability_counts.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import parity_workloads as pw  # noqa: E402


def main():
    lines = ["# Oracle stability counts of the parity workloads (oracle.c classifier).",
             "# Written by tests/golden/write_stability_counts.py; one JSON record per workload.",
             "# cases: stable / envelope / nonfinite (required class) / unchecked;",
             "# individuals: fit_strict / fit_envelope / fit_inf / fit_partial (tests/_parity.py)."]
    for name in pw.WORKLOADS:
        lines.append(json.dumps(pw.summary(name)))
    with open(os.path.join(HERE, "stability_counts.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
