"""Write tests/golden/shock_states.json: upstream and downstream states of the standing
shocks used as inputs, from the oracle's dense-gas Rankine-Hugoniot solver.

Calls only oracle/ (and the seeded parameter draws in workloads/).  Run from the
repository root:  python tests/golden/make_shock_states.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import physics  # noqa: E402
import workloads  # noqa: E402


def main():
    states = {}
    for mach in (2.0, 3.0):
        st = physics.shock_states(mach, 0.3)
        states[f"M{mach:g}_El0.3"] = st
    batch = {}
    for d in workloads.batch_draws():
        if d["kind"] != "shock":
            continue
        st = physics.shock_states(d["mach"], d["denseness"])
        batch[str(d["index"])] = dict(st, mach=d["mach"], denseness=d["denseness"])
    extra = {}
    # every closure draw gets its states (its kind depends on the sweep's size)
    for key, draws in (("closure", workloads.closure_draws(256)),
                       ("closure_held_out", workloads.closure_held_out())):
        extra[key] = {}
        for d in draws:
            if d["mach"] <= 1.0:
                continue
            st = physics.shock_states(d["mach"], d["denseness"])
            extra[key][str(d["index"])] = dict(st, mach=d["mach"], denseness=d["denseness"])
    out = {"comment": "dense-gas Rankine-Hugoniot end states, T1 + T2 = 2 scaling; written "
                      "by tests/golden/make_shock_states.py from oracle.physics",
           "states": states, "batch": batch, **extra}
    with open(os.path.join(HERE, "shock_states.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
