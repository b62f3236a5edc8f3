"""Launch shapes measured on an MI355X for the benchmark meshes (a data table, no arithmetic).

The library's autotuner (mm_plan_autotune) picks per-pass launch shapes on the
device.  Its picks for the benchmark meshes are kept in tuned_shapes.json so
that the benchmark, the full-size parity tests and the profiling runs all launch
the same kernel instantiations; mm_plan_set_shapes validates every entry against
the plan, so a stale entry fails loudly instead of launching a bad shape.
Keys: "<nx>x<ny>x<nz> <precision>".
"""
import json
import os

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_shapes.json")


def key(mesh, prec):
    return "%dx%dx%d %s" % (int(mesh[0]), int(mesh[1]), int(mesh[2]), prec)


def table(path=PATH):
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def lookup(mesh, prec, path=PATH):
    """The stored shapes (a dict as Plan.shapes() returns) or None."""
    return table(path).get(key(mesh, prec))


def store(mesh, prec, shapes, path=PATH):
    d = table(path)
    d[key(mesh, prec)] = {k: int(v) for k, v in shapes.items()}
    with open(path, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
        fh.write("\n")
