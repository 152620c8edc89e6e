"""Writes the stored expected values under tests/golden/ that are not the
paper's own numbers.  Calls only the CPU oracle and the seeded workload
generators.

    python tests/golden/make_golden.py
"""
import json
import os
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2605_24408_amd import workloads as W  # noqa: E402


def n12_optimum():
    """Exact minimum of Eq. 1 for the N=12 grid workload, by exhaustive
    enumeration of all 12! permutations (split on the facility at location 0)."""
    inst = W.config_n12()
    oracle.lib()
    with ThreadPoolExecutor(max_workers=os.cpu_count() or 4) as ex:
        res = list(ex.map(lambda f: oracle.brute_min(inst.D, inst.F, first=f), range(inst.N)))
    best = min(res, key=lambda t: t[0])
    return {"_source": "exhaustive enumeration of all 12! permutations with the CPU oracle "
                       "(tests/golden/make_golden.py)",
            "workload": inst.name, "optimum": int(best[0]),
            "argmin_perm": [int(v) for v in best[1]],
            "per_first_facility_min": [int(r[0]) for r in res]}


if __name__ == "__main__":
    out = n12_optimum()
    with open(os.path.join(HERE, "qap_n12_optimum.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)
