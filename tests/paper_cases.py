"""Map the golden-table entries to (box, density, closed-form potential)."""
import json
import os

import workloads as W
from oracle import analytic as A

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


def load():
    with open(GOLDEN) as f:
        return json.load(f)


def case(entry):
    n = entry["n"]
    box = W.Box(tuple(entry["a"]), tuple(entry["b"]), (n, n, n))
    p = entry["params"]
    kind = entry["density"]
    if kind == "gaussian":
        return box, W.paper_gaussian(box, p["sigma"]), A.gaussian(box, p["sigma"])
    if kind == "two_gaussians":
        return (box, W.paper_two_gaussians(box, p["d"], p["s1"], p["s2"]),
                A.two_gaussians(box, p["d"], p["s1"], p["s2"]))
    if kind == "bump":
        return box, W.paper_bump(box, p["d"], p["R"]), A.bump(box, p["d"], p["R"])
    if kind == "anisotropic":
        return box, W.paper_anisotropic(box, p["sig"]), A.anisotropic(box, p["sig"])
    if kind == "oscillating":
        return (box, W.paper_oscillating(box, p["sigma"], p["omega"]),
                A.oscillating(box, p["sigma"], p["omega"]))
    raise KeyError(kind)


def name(entry):
    return f"T{entry['table']}-{entry['density']}-{entry['n']}"
