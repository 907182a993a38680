"""Readers of the fixtures under tests/golden/ (values printed in the paper
or in a cited textbook; each file states its source)."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                yield line.split()


def table1():
    """{"alpha": .., "beta": .., "eta": ..} of Table I."""
    return {k: float(v) for k, v in _lines("table1_imex_ssp3_433.txt")}


def sod_star():
    return {k: float(v) for k, v in _lines("sod_exact_star_state.txt")}


def riemann2d():
    """{11: {"states": (Q1..Q4 as (rho, ux, uy, P)), "t_end": t, "rho_range": (lo, hi)}, 12: ..}"""
    out = {}
    for tok in _lines("riemann2d_c11_c12.txt"):
        c = int(tok[0][1:])
        e = out.setdefault(c, {"states": [None] * 4})
        if tok[1].startswith("Q"):
            e["states"][int(tok[1][1]) - 1] = tuple(float(x) for x in tok[2:6])
        elif tok[1] == "t_end":
            e["t_end"] = float(tok[2])
        elif tok[1] == "rho_range":
            e["rho_range"] = (float(tok[2]), float(tok[3]))
    for e in out.values():
        e["states"] = tuple(e["states"])
    return out
