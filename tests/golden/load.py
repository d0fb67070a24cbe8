"""Reader for the hand-derived worked examples in this folder."""
import glob
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load(path):
    case = {"name": os.path.basename(path)}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            if key == "algo":
                case["algo"] = vals[0]
            elif key in ("w", "M"):
                case[key] = int(vals[0])
            elif key == "bytes":
                case["data"] = np.array([int(v, 10) for v in vals], np.uint8)
            elif key == "hex":
                case["data"] = np.array([int(v, 16) for v in vals], np.uint8)
            elif key == "cuts":
                case["cuts"] = [int(v) for v in vals]
    return case


def all_cases():
    return [load(p) for p in sorted(glob.glob(os.path.join(HERE, "*.txt")))]
