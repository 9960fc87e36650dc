"""Readers for the hand-derived text fixtures under tests/golden/."""

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for raw in f:
            s = raw.strip()
            if s and not s.startswith("#"):
                yield s


def read_cases(name):
    """Blocks of 'case <id>', 'input' grid, 'expect' grid."""
    cases, cur, section = {}, None, None
    for s in _lines(name):
        if s.startswith("case "):
            cur = {"input": [], "expect": []}
            cases[s.split()[1]] = cur
            section = None
        elif s in ("input", "expect"):
            section = s
        else:
            cur[section].append([float(v) for v in s.split()])
    return {k: (np.array(v["input"]), np.array(v["expect"])) for k, v in cases.items()}


def read_pipeline(name):
    """Scalar parameters, 'input' / 'mask' / 'clean' grids and an 'n_new' row."""
    out, section = {"grids": {}}, None
    for s in _lines(name):
        tok = s.split()
        if tok[0] in ("input", "mask", "clean") and len(tok) == 1:
            section = tok[0]
            out["grids"][section] = []
        elif tok[0] == "n_new":
            out["n_new"] = [int(v) for v in tok[1:]]
        elif len(tok) == 2 and not tok[0][0].isdigit():
            out[tok[0]] = float(tok[1])
        else:
            out["grids"][section].append([float(v) for v in tok])
    out["grids"] = {k: np.array(v) for k, v in out["grids"].items()}
    return out


def read_pipeline_cases(name):
    """Several 'case <id>' blocks, each in read_pipeline's format."""
    blocks, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for raw in f:
            s = raw.strip()
            if s.startswith("case "):
                cur = s.split()[1]
                blocks[cur] = []
            elif cur is not None:
                blocks[cur].append(raw)
    return {k: _parse_pipeline(v) for k, v in blocks.items()}


def _parse_pipeline(lines):
    out, section = {"grids": {}}, None
    for raw in lines:
        s = raw.strip()
        if not s or s.startswith("#"):
            continue
        tok = s.split()
        if tok[0] in ("input", "mask", "clean") and len(tok) == 1:
            section = tok[0]
            out["grids"][section] = []
        elif tok[0] == "n_new":
            out["n_new"] = [int(v) for v in tok[1:]]
        elif len(tok) == 2 and not tok[0][0].isdigit():
            out[tok[0]] = float(tok[1])
        else:
            out["grids"][section].append([float(v) for v in tok])
    out["grids"] = {k: np.array(v) for k, v in out["grids"].items()}
    return out
