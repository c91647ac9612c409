"""Operation counts of the method per traced photon, from the oracle's counting build
(count.cpp) -- TEST AND MEASUREMENT INFRASTRUCTURE ONLY.

Traces a sample of photons of a scene through the counting build and writes, per stage (sky,
optics, sensor) and per photon outcome (status @ deciding surface), the mean number of FP64
additions/subtractions, multiplications, divisions, square roots and transcendental functions,
Philox blocks and screen bytes read.  The benchmark combines these means with the GPU launch's
own outcome counts to get the algorithmic work of each kernel.

    python -m oracle.count_ops --scene full --photons 200000 --out profiles/oracle_op_counts_full.json
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import subprocess
import sys
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "liborc_count.so")
STAGES = ("sky", "optics", "sensor")
FIELDS = ("add", "mul", "div", "sqrt", "trans", "philox", "gather_bytes")
FLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
         "-fvisibility=hidden", "-Wall", "-Wno-unused-function"]


def build() -> str:
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["g++", *FLAGS, "-o", tmp, os.path.join(_HERE, "count.cpp")])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("phx_oracle.c", "phx_oracle.h", "count.cpp"):
        h.update(open(os.path.join(_HERE, f), "rb").read())
    return h.hexdigest()[:16]


def count(scene, photons, threads=8):
    """Events and per-photon counts [n][3 stages][7 fields] of photons (indices of source 0)."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import oracle as O
    if not os.path.exists(LIB_PATH):
        build()
    L = C.CDLL(LIB_PATH)
    L.orc_count_trace_list.argtypes = [C.POINTER(O.Scene), C.c_int32, C.c_void_p, C.c_uint64,
                                       C.c_void_p, C.c_void_p]
    L.orc_count_trace_list.restype = C.c_int
    orc = O.Oracle(scene)      # the oracle library prepares the scene (tables, transforms)
    ph = np.ascontiguousarray(photons, np.uint64)
    ev = np.zeros(len(ph), O.EVENT_DTYPE)
    cnt = np.zeros((len(ph), len(STAGES), len(FIELDS)), np.uint64)
    parts = np.array_split(np.arange(len(ph)), max(1, threads))

    def run(idx):
        if len(idx) == 0:
            return
        a, b = int(idx[0]), int(idx[-1]) + 1
        rc = L.orc_count_trace_list(C.byref(orc.sc), 0, ph[a:b].ctypes.data, b - a,
                                    ev[a:b].ctypes.data, cnt[a:b].ctypes.data)
        assert rc == 0
    ths = [threading.Thread(target=run, args=(p,)) for p in parts]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    return ev, cnt


def table(ev, cnt):
    """Mean counts per stage and field, over all photons and per outcome 'STATUS@surface'."""
    import oracle as O

    def means(sel):
        m = cnt[sel].astype(np.float64).mean(axis=0)
        return {st: {f: float(m[i, j]) for j, f in enumerate(FIELDS)} for i, st in
                enumerate(STAGES)}
    out = {"all": dict(n=int(len(ev)), **means(np.ones(len(ev), bool)))}
    keys = sorted(set(zip(ev["status"].tolist(), ev["surface"].tolist())))
    for st, sf in keys:
        sel = (ev["status"] == st) & (ev["surface"] == sf)
        out[f"{O.STATUS[st]}@{sf}"] = dict(n=int(sel.sum()), **means(sel))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scene", default="full")
    ap.add_argument("--photons", type=int, default=200000)
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "oracle_op_counts_full.json"))
    args = ap.parse_args()
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from paper_1504_06570_amd.scene import configs as Cfg
    build()
    scene = Cfg.CONFIGS[args.scene]()
    ev, cnt = count(scene, np.arange(args.photons, dtype=np.uint64), args.threads)
    rec = {
        "what": "mean operations per photon of the oracle's counting build, per stage and per "
                "outcome (status@deciding surface); FP64 add/sub, mul, div, sqrt, "
                "transcendental each one operation; Philox blocks; screen bytes read",
        "command": "python -m oracle.count_ops " + " ".join(
            f"--{k} {v}" for k, v in (("scene", args.scene), ("photons", args.photons))),
        "scene": args.scene,
        "photons": args.photons,
        "oracle_hash": source_hash(),
        "stages": list(STAGES),
        "fields": list(FIELDS),
        "by_outcome": table(ev, cnt),
    }
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    a = rec["by_outcome"]["all"]
    print(json.dumps({st: a[st] for st in STAGES}))


if __name__ == "__main__":
    main()
