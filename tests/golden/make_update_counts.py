"""Write tests/golden/update_counts.json: exact A-updates (Joseph samples
whose bilinear support touches the volume; for the line-intersection
projector, ray-voxel segments) and B-updates (voxel-view pairs) per workload
geometry, counted by the FP64 oracle only.

    python tests/golden/make_update_counts.py
"""

import dataclasses
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth import workloads  # noqa: E402


def main():
    out = {}
    for name, desc in [("w1", workloads.w1_geometry()), ("w2", workloads.w2_geometry()),
                       ("w3", workloads.w3_geometry())]:
        out[name] = {"A_updates": oracle.count_A_updates(desc),
                     "B_updates": oracle.count_B_updates(desc),
                     "n_vox": desc.n_vox, "n_rays": desc.n_rays}
        print(name, out[name], flush=True)
    g3s = dataclasses.replace(workloads.w3_geometry(), projector=1)
    out["w3_siddon"] = {"A_updates": oracle.count_A_updates(g3s)}
    print("w3_siddon", out["w3_siddon"], flush=True)
    gp = workloads.paper_geometry()
    out["paper"] = {"A_updates": oracle.count_A_updates(gp), "B_updates": oracle.count_B_updates(gp),
                    "n_vox": gp.n_vox, "n_rays": gp.n_rays}
    print("paper", out["paper"], flush=True)
    w5 = [oracle.count_A_updates(d) for d, _, _ in workloads.w5_slices()]
    out["w5"] = {"A_updates": int(sum(w5)),
                 "B_updates": int(sum(d.n_vox * d.n_views for d, _, _ in workloads.w5_slices()))}
    with open(os.path.join(HERE, "update_counts.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
