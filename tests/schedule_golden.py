"""Reader for the worked schedule examples under tests/golden/ (no method
arithmetic)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "schedule_worked_examples.txt")


GOLDEN_REFINED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                              "schedule_refined_examples.txt")


def load_examples(path=GOLDEN):
    out = []
    cur = None
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(" ")
            if key == "name":
                cur = {"name": rest, "waves": []}
            elif key == "grid":
                cur["hb"], cur["wb"] = map(int, rest.split())
            elif key == "lost":
                cur["lost"] = np.array([int(c) for c in rest], np.uint8).reshape(cur["hb"], cur["wb"])
            elif key == "outside":
                cur["outside"] = int(rest)
            elif key == "unknown":
                cur["unknown"] = np.array([int(t) for t in rest.split()],
                                          np.int32).reshape(cur["hb"], cur["wb"])
            elif key == "wave":
                cur["waves"].append([int(t) for t in rest.split()])
            elif key == "end":
                out.append(cur)
                cur = None
    return out
