"""Shared test plumbing: converts fixture schemas for libdc and compares
planner/oracle object tables. No method arithmetic lives here."""
import numpy as np


def dc_schema(types):
    from paper_1906_01128_amd import dc
    return dc.Schema(types)


def plan_of(t, align=64, follow=None):
    from paper_1906_01128_amd import dc
    schema = dc_schema(t.types)
    return dc.Plan(schema, t.root_type, t.roots, align=align, follow=follow)


def same_objects(plan_objs, oracle_objs):
    """Host address, offset, bytes, count, kind and type of every object."""
    assert len(plan_objs) == len(oracle_objs)
    for name in ("host", "off", "bytes", "count", "kind", "type"):
        a = plan_objs[name].astype(np.uint64)
        b = oracle_objs[name].astype(np.uint64)
        # types of primitive arrays are not meaningful
        if name == "type":
            keep = oracle_objs["kind"] == 0
            a, b = a[keep], b[keep]
        assert np.array_equal(a, b), f"object field {name} differs"
