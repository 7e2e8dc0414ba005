"""Loader for the hand-built scenes under tests/golden/ (closed-form expectations)."""
import glob
import json
import math
import os

import numpy as np

from synth import PRED_NAMES, QueryBatch, Scene

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _sig(u):
    return 1.0 / (1.0 + math.exp(-u))


_NS = {"exp": math.exp, "log": math.log, "sqrt": math.sqrt, "sig": _sig}


def evaluate(expr: str) -> float:
    return float(eval(expr, {"__builtins__": {}}, dict(_NS)))


def load(path):
    with open(path) as f:
        g = json.load(f)
    objs = g["objects"]
    d = int(g["d"])
    scene = Scene(
        desc=np.asarray([o["desc"] for o in objs], np.float32).reshape(len(objs), d),
        center=np.asarray([o["center"] for o in objs], np.float32).reshape(len(objs), 3),
        extent=np.full((len(objs), 3), 0.5, np.float32),
        ids=np.asarray([o["id"] for o in objs], np.uint32),
        cls=np.asarray([o["cls"] for o in objs], np.int32),
        view_right=np.asarray(g["view_right"], np.float32),
        centroids=np.zeros((1, d), np.float32),
    )
    queries = []
    for q in g["queries"]:
        rels = q["relations"]
        qb = QueryBatch(
            target=np.asarray([q["target"]], np.float32),
            target_cls=np.asarray([q["target_cls"]], np.int32),
            rel_off=np.asarray([0, len(rels)], np.int32),
            rel_pred=np.asarray([PRED_NAMES.index(r[0]) for r in rels], np.int32),
            rel_anchor=np.asarray([r[1] for r in rels], np.float32).reshape(len(rels), d),
            planted=np.zeros(1, np.int64),
        )
        queries.append((qb, q))
    return g, scene, queries


def all_paths():
    return sorted(glob.glob(os.path.join(GOLDEN_DIR, "*.json")))
