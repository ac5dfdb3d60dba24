"""Python face of the query server: induced-subgraph triangle counts and
average clustering coefficients over a resident graph, with memory-based
admission and continuous batching (all in the native library)."""
import ctypes

import numpy as np
import torch

from . import _native as N
from .graph import _ptr

TRICC_EBUSY = N.TRICC_EBUSY


class ServerError(N.TriccError):
    pass


def _check(rc, what):
    if rc != N.TRICC_OK:
        e = ServerError.__new__(ServerError)
        e.status = rc
        RuntimeError.__init__(e, f"{what}: {N.status_str(rc)} ({rc}): "
                                 f"{N.lib().tricc_server_last_error().decode()}")
        raise e


class Server:
    """``graph``: a built :class:`Graph` (kept resident). ``workspace_bytes``
    of device memory are split into ``slots`` equal slices; the same amount is
    the admission budget."""

    def __init__(self, graph, workspace_bytes, slots=2, max_batch_queries=256):
        self.graph = graph
        self.ws = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=graph.device)
        self._h = ctypes.c_void_p()
        with torch.cuda.device(graph.device):
            rc = N.lib().tricc_server_create(graph._h, _ptr(self.ws), self.ws.numel(), slots, max_batch_queries,
                                             ctypes.byref(self._h))
        _check(rc, "tricc_server_create")

    def set_tuning(self, tuning):
        t = N.BatchTuning.from_dict(tuning) if isinstance(tuning, dict) else tuning
        _check(N.lib().tricc_server_set_tuning(self._h, ctypes.byref(t)), "tricc_server_set_tuning")

    def now(self):
        return N.lib().tricc_server_now(self._h)

    def query_bytes(self, nodes):
        a = np.ascontiguousarray(nodes, dtype=np.int32)
        return N.lib().tricc_server_query_bytes(self._h, a.ctypes.data_as(ctypes.c_void_p), a.size)

    def submit(self, qid, nodes, t_arrival=None):
        """Returns TRICC_OK or TRICC_EBUSY; raises on other errors."""
        a = np.ascontiguousarray(nodes, dtype=np.int32)
        t = self.now() if t_arrival is None else float(t_arrival)
        rc = N.lib().tricc_server_submit(self._h, int(qid), a.ctypes.data_as(ctypes.c_void_p), a.size, t)
        if rc == N.TRICC_EBUSY:
            return rc
        _check(rc, "tricc_server_submit")
        return rc

    def poll(self, cap=4096):
        buf = (N.QueryResult * cap)()
        n = ctypes.c_int32()
        _check(N.lib().tricc_server_poll(self._h, buf, cap, ctypes.byref(n)), "tricc_server_poll")
        return [buf[i].as_dict() for i in range(n.value)]

    def drain(self):
        _check(N.lib().tricc_server_drain(self._h), "tricc_server_drain")

    def stats(self):
        w, f, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
        _check(N.lib().tricc_server_stats(self._h, ctypes.byref(w), ctypes.byref(f), ctypes.byref(b)),
               "tricc_server_stats")
        return {"waiting": w.value, "in_flight": f.value, "outstanding_bytes": b.value}

    def close(self):
        if self._h:
            N.lib().tricc_server_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
