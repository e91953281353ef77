"""Readers for the paper fixtures under tests/golden (values printed in the paper)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _sections(name):
    out, cur, tags = {}, None, {}
    for line in open(os.path.join(GOLDEN, name)):
        s = line.strip()
        if not s:
            continue
        if s.startswith("#"):
            parts = s[1:].split()
            if len(parts) == 1:
                cur = parts[0]
                out[cur] = []
            elif parts and parts[0].isupper() and all(p.lstrip("-").replace(".", "").isdigit() for p in parts[1:]):
                tags[parts[0]] = [float(p) for p in parts[1:]]
            continue
        out.setdefault(cur, []).append([float(v) for v in s.split()])
    return {k: np.array(v) for k, v in out.items()}, tags


def refine_example():
    s, _ = _sections("refine_example.txt")
    return s["T"].astype(int), s["C"]


def nodes2edge_example():
    s, tags = _sections("nodes2edge_example.txt")
    tets = np.array(tags["TETS"], dtype=int).reshape(-1, 4)
    return tets, s[None].astype(int)


def faces_listing1():
    s, tags = _sections("faces_listing1.txt")
    return s[None].astype(int), np.array(tags["TET5"], dtype=int)


def counts_tables():
    s, _ = _sections("counts_tables.txt")
    return s[None].astype(np.int64)


def table4_errors():
    """rows: level, Y-error, Y-order, h-error, h-order (Table 4)"""
    return np.loadtxt(os.path.join(GOLDEN, "table4_errors.txt"))
