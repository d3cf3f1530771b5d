"""The CPU oracle over disjoint packet-id ranges in worker processes, for
parity checks of whole launches (test infrastructure only).

Every packet's history depends only on its own random stream, so an
iteration's raw tallies are the sums of the tallies of any partition of its
packet ids.  Each worker is a fresh interpreter that rebuilds the workload
from its name, runs the oracle on its id range and saves its raw tallies;
the parent adds them up.  Workers start as child processes (never by
replacing a process that has touched the GPU).

    run_split("config2", {}, T_inner, ids, procs)  -> raw dict as oracle.run
"""
from __future__ import annotations

import json
import os
import subprocess
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def workload(name: str, kwargs: dict):
    """The workload a worker rebuilds: a generator of workloads.py by name."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from paper_1401_5469_amd import workloads as W
    return getattr(W, name)(**kwargs)


def default_procs() -> int:
    # the GPU machine gives one GPU 16 host cores whatever os.cpu_count() says
    return max(1, min(16, os.cpu_count() or 1))


def run_split(name: str, kwargs: dict, T_inner: float, ids, procs: int | None = None,
              iteration: int = 0, want_packets: bool = True, want_jblue: bool = True):
    """Raw oracle tallies of packet ids `ids` (sorted uint64), split over
    worker processes: the sums of the workers' J, nu-bar, J_blue, spectrum
    and luminosity tallies and counters, and the per-packet records in id
    order."""
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    procs = procs or default_procs()
    parts = [p for p in np.array_split(ids, procs) if p.size]
    with tempfile.TemporaryDirectory(prefix="oracle_pool_") as tmp:
        workers = []
        for k, part in enumerate(parts):
            ids_path = os.path.join(tmp, f"ids{k}.npy")
            np.save(ids_path, part)
            spec = dict(name=name, kwargs=kwargs, T=T_inner, iteration=iteration,
                        ids=ids_path, out=os.path.join(tmp, f"out{k}.npz"),
                        packets=want_packets, jblue=want_jblue)
            workers.append(subprocess.Popen([sys.executable, os.path.abspath(__file__),
                                             json.dumps(spec)]))
        codes = [w.wait() for w in workers]
        if any(codes):
            raise RuntimeError(f"oracle workers failed: {codes}")
        outs = [np.load(os.path.join(tmp, f"out{k}.npz")) for k in range(len(parts))]
        raw = {}
        for key in ("J_raw", "nubar_raw", "spec_raw", "L_raw", "counters"):
            raw[key] = np.sum([o[key] for o in outs], axis=0)
        raw["jblue_raw"] = (np.sum([o["jblue_raw"] for o in outs], axis=0)
                            if want_jblue else None)
        raw["packets"] = (np.concatenate([o["packets"] for o in outs])
                          if want_packets else None)
    from oracle import oracle as O
    raw["counters"] = {k: int(v) for k, v in zip(O.COUNTER_NAMES, raw["counters"])}
    return raw


def _worker(spec: dict) -> None:
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from oracle import oracle as O
    w = workload(spec["name"], spec["kwargs"])
    ids = np.load(spec["ids"])
    r = O.run(w.model, spec["T"], w.n_packets, iteration=spec["iteration"], packet_ids=ids,
              want_jblue=spec["jblue"], want_packets=spec["packets"])
    counters = np.array([r["counters"][k] for k in O.COUNTER_NAMES], dtype=np.uint64)
    out = dict(J_raw=r["J_raw"], nubar_raw=r["nubar_raw"], spec_raw=r["spec_raw"],
               L_raw=r["L_raw"], counters=counters)
    if spec["jblue"]:
        out["jblue_raw"] = r["jblue_raw"]
    if spec["packets"]:
        out["packets"] = r["packets"]
    np.savez(spec["out"], **out)


if __name__ == "__main__":
    _worker(json.loads(sys.argv[1]))
