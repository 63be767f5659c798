"""Pointer-graph decoding for the pins: reads a host tree straight from host
memory, or a deep-copied buffer straight from its bytes, using only the struct
descriptions. Independent of both the oracle and the HIP library."""
from __future__ import annotations

import ctypes
import itertools
import struct
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

ELEM = {"f32": 4, "f64": 8, "i32": 4, "i64": 8, "u8": 1}


def elem_size(types, kind, type_idx):
    return types[type_idx].size if kind == "struct" else ELEM[kind]


def count_of(fld, elem_bytes: bytes) -> int:
    if fld.count_offset < 0:
        return fld.fixed_count
    raw = elem_bytes[fld.count_offset: fld.count_offset + fld.count_bytes]
    n = int.from_bytes(raw, "little", signed=True)
    assert n >= 0
    return n * fld.count_mult


@dataclass
class Node:
    key: int              # host address or buffer address
    kind: str
    type: int
    count: int
    data: bytes           # object bytes with pointer slots zeroed
    edges: List[Tuple[int, int, int]] = field(default_factory=list)  # (elem, field idx, target key)


def _decode(types, root_type, roots, read, translate=lambda p: p):
    """Generic decoder. read(addr, n) returns bytes at addr; translate maps a
    stored pointer to the address `read` understands."""
    nodes: Dict[int, Node] = {}
    order: List[int] = []
    stack = []
    for r in roots:
        if r not in nodes:
            nodes[r] = Node(r, "struct", root_type, 1, b"")
            stack.append(r)
            order.append(r)
    while stack:
        k = stack.pop()
        nd = nodes[k]
        size = elem_size(types, nd.kind, nd.type) * nd.count
        raw = bytearray(read(translate(k), size))
        if nd.kind == "struct":
            t = types[nd.type]
            for e in range(nd.count):
                eb = bytes(raw[e * t.size:(e + 1) * t.size])
                for fi, fld in enumerate(t.fields):
                    p = int.from_bytes(eb[fld.offset: fld.offset + 8], "little")
                    raw[e * t.size + fld.offset: e * t.size + fld.offset + 8] = b"\0" * 8
                    if p == 0:
                        continue
                    n = count_of(fld, eb)
                    ptype = fld.type if fld.kind == "struct" else 0
                    nd.edges.append((e, fi, p))
                    if p not in nodes:
                        nodes[p] = Node(p, fld.kind, ptype, n, b"")
                        stack.append(p)
                        order.append(p)
                    else:
                        o = nodes[p]
                        assert (o.kind, o.type, o.count) == (fld.kind, ptype, n)
        nd.data = bytes(raw)
    return nodes, order


def host_graph(types, root_type, roots):
    return _decode(types, root_type, roots, lambda a, n: ctypes.string_at(a, n) if n else b"")


def arena_graph(types, root_type, arena: bytes, base: int, root_offsets):
    roots = [base + o for o in root_offsets]
    return _decode(types, root_type, roots, lambda a, n: bytes(arena[a - base: a - base + n]))


def signature(nd: Node):
    return (nd.kind, nd.type, nd.count, nd.data)


def preserving_bijections(g1: Dict[int, Node], g2: Dict[int, Node], limit=8):
    """Every bijection g1 -> g2 that preserves kind, type, count, non-pointer
    bytes and every labelled edge. Brute force; for graphs of at most `limit`
    nodes."""
    k1 = sorted(g1)
    k2 = sorted(g2)
    assert len(k1) == len(k2) and len(k1) <= limit
    out = []
    for perm in itertools.permutations(k2):
        m = dict(zip(k1, perm))
        if any(signature(g1[a]) != signature(g2[m[a]]) for a in k1):
            continue
        ok = True
        for a in k1:
            e1 = sorted((e, f, m[t]) for e, f, t in g1[a].edges)
            e2 = sorted(g2[m[a]].edges)
            if e1 != e2:
                ok = False
                break
        if ok:
            out.append(m)
    return out


def depths(g: Dict[int, Node], roots) -> Dict[int, int]:
    """Breadth-first hop count from the nearest root."""
    d = {}
    frontier = list(dict.fromkeys(roots))
    for r in frontier:
        d[r] = 0
    while frontier:
        nxt = []
        for k in frontier:
            for _, _, t in g[k].edges:
                if t not in d:
                    d[t] = d[k] + 1
                    nxt.append(t)
        frontier = nxt
    return d


def pointer_slots(types, objects, arena: bytes):
    """(slot offset, stored value) for every pointer slot of every struct
    object in a buffer, from a table of (off, count, kind, type)."""
    out = []
    for o in objects:
        if o["kind"] != 0:
            continue
        t = types[int(o["type"])]
        for e in range(int(o["count"])):
            for fld in t.fields:
                s = int(o["off"]) + e * t.size + fld.offset
                out.append((s, int.from_bytes(arena[s:s + 8], "little")))
    return out
