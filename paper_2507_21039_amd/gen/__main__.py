"""Write the generated process headers: python -m paper_2507_21039_amd.gen [outdir]."""
import json
import os
import sys

from . import diagrams, emit

PROCESSES = {
    # name: (struct name, number of final-state gluons, label)
    "ggtt": ("P_ggtt", 0, "g g -> t tbar"),
    "ggttg": ("P_ggttg", 1, "g g -> t tbar g"),
    "ggttgg": ("P_ggttgg", 2, "g g -> t tbar g g"),
}


def generate(outdir: str, names=None) -> dict:
    os.makedirs(outdir, exist_ok=True)
    infos = {}
    hdr, info = emit.emit_eemumu("P_eemumu")
    todo = [("eemumu", hdr, info)]
    for key, (struct, ng, label) in PROCESSES.items():
        if names and key not in names:
            continue
        g = diagrams.build_graph(ng)
        hdr, info = emit.emit_qcd(struct, g, label)
        todo.append((key, hdr, info))
    for key, hdr, info in todo:
        path = os.path.join(outdir, f"{key}.h")
        old = open(path).read() if os.path.exists(path) else None
        if old != hdr:
            with open(path, "w") as f:
                f.write(hdr)
        infos[key] = {k: v for k, v in info.items() if k != "numerators"}
    with open(os.path.join(outdir, "processes.json"), "w") as f:
        json.dump(infos, f, indent=1, sort_keys=True)
    return infos


if __name__ == "__main__":
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.dirname(__file__)), "csrc", "procs")
    for k, v in generate(out).items():
        print(k, v)
