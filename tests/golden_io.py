"""Reader for the hand-worked fixtures in tests/golden (plain text, one key per line)."""
import glob
import os


def load(path):
    case = {"file": os.path.basename(path), "planes": [], "expect_planes": []}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            if key == "plane":
                case["planes"].append([int(v) for v in vals])
            elif key == "expect_plane":
                case["expect_planes"].append([int(v) for v in vals])
            elif key in ("op",):
                case[key] = vals[0]
            elif key == "input":
                case["input"] = vals
            else:
                case[key] = [int(v) for v in vals]
    return case


def load_all(golden_dir):
    return [load(p) for p in sorted(glob.glob(os.path.join(golden_dir, "*.txt")))]
