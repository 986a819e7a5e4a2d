"""Hand-derived fixtures for the oracle pins (see the comments in each file)."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def load_splits(name="splits_1d.txt"):
    """Parse the hand-traced split records into a list of dicts."""
    cases, cur = [], None
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(" ")
            if key == "case":
                cur = {"case": rest}
                cases.append(cur)
                continue
            vals = rest.split()
            if key in ("points", "centres"):
                cur[key] = [float(v) for v in vals]
            else:
                cur[key] = [int(v) for v in vals]
    return cases
