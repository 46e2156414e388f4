"""Writes cfg0_events.json: the CPU oracle's vote totals and peak lists for workload-0 events.

Calls only the oracle (and the seeded event generator); the stored values are regression
fixtures for the oracle itself. Run from the repository root: python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_1507_03074_amd import synth  # noqa: E402


def main():
    spec = synth.WORKLOADS[0].grid
    g = oracle.OracleGrid(*spec.as_tuple())
    events = []
    for e in range(20):
        ev = synth.make_event(0, e)
        M, votes = oracle.fill(g, ev.x, ev.y, ev.z)
        cells, vv, n = oracle.peaks(g, M)
        events.append({"event": e, "n_hits": ev.n, "votes": votes,
                       "peaks": [[int(c), int(v)] for c, v in zip(cells, vv)]})
    out = {"workload": synth.WORKLOADS[0].name, "grid": list(spec.as_tuple()),
           "written_by": "tests/golden/make_golden.py (oracle only)", "events": events}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg0_events.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
