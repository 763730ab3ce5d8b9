"""ORACLE (test infrastructure only): is a returned mapping a valid common
induced subgraph (paper Sec. II.A)?  Checks that pairs are in range, the map
is injective on both sides, labels agree, and every ordered pair of mapped
vertices agrees on adjacency."""
from __future__ import annotations


def mapping_errors(G: dict, H: dict, pairs) -> list:
    errs = []
    gs = [p[0] for p in pairs]
    hs = [p[1] for p in pairs]
    for g, h in pairs:
        if not (0 <= g < G["n"]) or not (0 <= h < H["n"]):
            errs.append(f"pair {(g, h)} out of range")
    if errs:
        return errs
    if len(set(gs)) != len(gs):
        errs.append("a G vertex is mapped twice")
    if len(set(hs)) != len(hs):
        errs.append("an H vertex is mapped twice")
    if G.get("label") is not None:
        for g, h in pairs:
            if G["label"][g] != H["label"][h]:
                errs.append(f"labels differ on {(g, h)}")
    for g1, h1 in pairs:
        for g2, h2 in pairs:
            if g1 == g2:
                continue
            if ((G["rows"][g1] >> g2) & 1) != ((H["rows"][h1] >> h2) & 1):
                errs.append(f"adjacency differs on {(g1, g2)} vs {(h1, h2)}")
    return errs


def is_valid(G: dict, H: dict, pairs) -> bool:
    return not mapping_errors(G, H, pairs)
