"""Python front end of the serving runtime (continuous batching in libscprop).

``Server`` wraps scp_server_*; ``run_stream`` replays a Poisson stream of
requests against it in wall-clock time and reports latency percentiles and
throughput.  All scheduling, admission and batching happen in the library.
"""
from __future__ import annotations

import ctypes as C
import sys
import time

import numpy as np
import torch

from ._lib import check, lib
from .api import _stream_ptr, marshal

STATE = {0: "queued", 1: "running", 2: "done", 3: "failed"}


class Server:
    ENGINES = {"auto": 0, "register": 1, "gather": 2}

    def __init__(self, hbm_budget_bytes, max_active=64, chunk_work=0.0, stream=None,
                 engine="register"):
        h = C.c_void_p()
        check(lib().scp_server_create(int(hbm_budget_bytes), int(max_active), float(chunk_work),
                                      _stream_ptr(stream), C.byref(h)))
        self.handle = h
        self.n_params = {}
        check(lib().scp_server_set_engine(self.handle, self.ENGINES[engine]))

    def submit(self, desc, want_grad):
        sd, keep = marshal(desc)
        cols = np.ascontiguousarray(np.asarray(desc["columns"], dtype=np.int64))
        rows = np.ascontiguousarray(np.asarray(desc["comp_rows"], dtype=np.int64))
        ccols = np.ascontiguousarray(np.asarray(desc["comp_cols"], dtype=np.int32))
        T = np.asarray(desc["target"], dtype=np.complex128)
        tgt = np.ascontiguousarray(np.stack([T.real, T.imag], axis=-1).reshape(-1))
        rid = C.c_int64()
        check(lib().scp_server_submit(
            self.handle, C.byref(sd), cols.ctypes.data_as(C.POINTER(C.c_int64)), len(cols),
            rows.ctypes.data_as(C.POINTER(C.c_int64)),
            ccols.ctypes.data_as(C.POINTER(C.c_int32)), len(rows),
            tgt.ctypes.data_as(C.POINTER(C.c_double)), int(bool(want_grad)), C.byref(rid)))
        n = sum(len(d["params"]) for d in desc["drives"]) + 3 * len(desc["modes"]) + \
            len(desc["couplings"])
        self.n_params[rid.value] = n
        return rid.value

    def step(self):
        a, q = C.c_int32(), C.c_int32()
        check(lib().scp_server_step(self.handle, C.byref(a), C.byref(q)))
        return a.value, q.value

    def result(self, rid):
        st, F, npar = C.c_int32(), C.c_double(), C.c_int32()
        ts, ta, td = C.c_double(), C.c_double(), C.c_double()
        g = (C.c_double * max(1, self.n_params.get(rid, 1)))()
        check(lib().scp_server_result(self.handle, rid, C.byref(st), C.byref(F), g, C.byref(npar),
                                      C.byref(ts), C.byref(ta), C.byref(td)))
        out = {"state": STATE[st.value], "F": F.value, "t_submit": ts.value,
               "t_admit": ta.value, "t_done": td.value}
        if st.value == 2 and npar.value:
            out["grad"] = np.array(g[: npar.value])
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().scp_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def request_bytes(desc, want_grad):
    """Device footprint the server reserves for a request."""
    sd, keep = marshal(desc)
    n = C.c_size_t()
    check(lib().scp_request_bytes(C.byref(sd), len(desc["columns"]), int(bool(want_grad)),
                                  C.byref(n)))
    return n.value


def drain(server, ids, timeout_s=600.0):
    """Step until every id has finished; returns their results."""
    t0 = time.perf_counter()
    pending = set(ids)
    res = {}
    while pending:
        server.step()
        for rid in list(pending):
            r = server.result(rid)
            if r["state"] in ("done", "failed"):
                res[rid] = r
                pending.discard(rid)
        if time.perf_counter() - t0 > timeout_s:
            raise TimeoutError(f"{len(pending)} requests unfinished")
    return res


def run_stream(requests, arrivals, hbm_budget_bytes, max_active=64, chunk_work=0.0,
               timeout_s=900.0, engine="register", progress_s=0.0):
    """Submit ``requests`` (descriptor dicts with a ``want_grad`` flag) at
    ``arrivals`` (seconds from start) and serve them; returns per-request
    latency (completion - arrival, wall clock) and summary statistics.
    progress_s > 0 prints a progress line to stderr at that interval."""
    srv = Server(hbm_budget_bytes, max_active, chunk_work, engine=engine)
    t_print = progress_s
    n = len(requests)
    ids = [None] * n
    sub_wall = [0.0] * n
    done_wall = {}
    nxt = 0
    t0 = time.perf_counter()
    pending = set()
    while len(done_wall) < n:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= now:
            ids[nxt] = srv.submit(requests[nxt], requests[nxt].get("want_grad", False))
            sub_wall[nxt] = time.perf_counter() - t0
            pending.add(nxt)
            nxt += 1
        if not pending:
            time.sleep(max(0.0, min(arrivals[nxt] - now, 0.01)))
            continue
        srv.step()
        tnow = time.perf_counter() - t0
        for i in list(pending):
            r = srv.result(ids[i])
            if r["state"] in ("done", "failed"):
                done_wall[i] = (tnow, r)
                pending.discard(i)
        if progress_s > 0 and tnow >= t_print:
            sys.stderr.write(f"[serve] {tnow:.0f} s: {len(done_wall)} of {n} done, "
                             f"{len(pending)} in flight\n")
            sys.stderr.flush()
            t_print = tnow + progress_s
        if tnow > timeout_s:
            raise TimeoutError("serving stream did not finish")
    lat = np.array([done_wall[i][0] - arrivals[i] for i in range(n)])
    total = max(d[0] for d in done_wall.values())
    work = sum(q["n_steps"] * (max(m["trunc"] for m in q["modes"]) ** len(q["modes"])) * len(q["columns"])
               for q in requests)
    failed = sum(1 for d in done_wall.values() if d[1]["state"] != "done")
    srv.close()
    return {"n": n, "failed": failed, "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
            "makespan_s": total, "requests_per_s": n / total,
            "steps_dim2_per_s": work / total, "results": {i: done_wall[i][1] for i in range(n)}}
