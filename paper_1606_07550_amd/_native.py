"""ctypes binding of ``libtricc.so`` (the C ABI in ``include/tricc.h``).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library. There is no fallback; if the library is missing the
import of :func:`lib` raises.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtricc.so")

TRICC_OK = 0
TRICC_EINVAL = 1
TRICC_ERANGE = 2
TRICC_ENOMEM = 3
TRICC_EHIP = 4
TRICC_EBUSY = 5
TRICC_EOVERFLOW = 6
NUM_BINS = 6


class TriccError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status}): {last_error()}")


class Tuning(ctypes.Structure):
    _fields_ = [("bin_limit", ctypes.c_int32 * (NUM_BINS - 1)),
                ("bin_variant", ctypes.c_int32 * NUM_BINS),
                ("min_side", ctypes.c_int32)]

    def as_dict(self):
        return {"bin_limit": list(self.bin_limit), "bin_variant": list(self.bin_variant),
                "min_side": self.min_side}

    @classmethod
    def from_dict(cls, d):
        t = cls()
        for i, v in enumerate(d["bin_limit"]):
            t.bin_limit[i] = int(v)
        for i, v in enumerate(d["bin_variant"]):
            t.bin_variant[i] = int(v)
        t.min_side = int(d.get("min_side", 0))
        return t


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m_raw", ctypes.c_int64), ("m", ctypes.c_int64),
                ("max_deg", ctypes.c_int64), ("max_outdeg", ctypes.c_int64),
                ("bin_count", ctypes.c_int64 * NUM_BINS), ("list_elems", ctypes.c_uint64),
                ("large_rows", ctypes.c_int64), ("bin_list_elems", ctypes.c_uint64 * NUM_BINS),
                ("bin_edges", ctypes.c_int64 * NUM_BINS), ("bin_in_items", ctypes.c_int64 * NUM_BINS),
                ("n_deg2", ctypes.c_int64), ("bin_kernel_bytes", ctypes.c_uint64 * NUM_BINS)]

    def as_dict(self):
        return {"n": self.n, "m_raw": self.m_raw, "m": self.m, "max_deg": self.max_deg,
                "max_outdeg": self.max_outdeg, "bin_count": list(self.bin_count),
                "list_elems": int(self.list_elems), "large_rows": self.large_rows,
                "bin_list_elems": [int(x) for x in self.bin_list_elems], "bin_edges": list(self.bin_edges),
                "bin_in_items": list(self.bin_in_items), "n_deg2": self.n_deg2,
                "bin_kernel_bytes": list(self.bin_kernel_bytes)}


class BatchTuning(ctypes.Structure):
    _fields_ = [("merge_limit", ctypes.c_int32), ("wave_limit", ctypes.c_int32),
                ("persist_variant", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

    @classmethod
    def from_dict(cls, d):
        return cls(int(d.get("merge_limit", 0)), int(d["wave_limit"]), int(d["persist_variant"]),
                   int(d["blocks_per_cu"]))


class BatchInfo(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_int32), ("total_nodes", ctypes.c_int64), ("total_pairs", ctypes.c_int64),
                ("m", ctypes.c_int64), ("max_outdeg", ctypes.c_int64), ("merge_nodes", ctypes.c_int64),
                ("wave_nodes", ctypes.c_int64),
                ("block_nodes", ctypes.c_int64), ("hub_nodes", ctypes.c_int64), ("grid", ctypes.c_int32),
                ("planned", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class QueryResult(ctypes.Structure):
    _fields_ = [("qid", ctypes.c_uint64), ("k", ctypes.c_int64), ("triangles", ctypes.c_uint64),
                ("avg_cc", ctypes.c_double), ("m", ctypes.c_int64), ("t_arrival", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double), ("batch_size", ctypes.c_int32),
                ("status", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_LIB = None

# name -> (restype, argtypes)
_P = ctypes.c_void_p
_SIGS = {
    "tricc_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "tricc_last_error": (ctypes.c_char_p, []),
    "tricc_version": (ctypes.c_int, []),
    "tricc_default_tuning": (ctypes.c_int, [ctypes.POINTER(Tuning)]),
    "tricc_variant_capacity": (ctypes.c_int, [ctypes.c_int]),
    "tricc_variant_count": (ctypes.c_int, []),
    "tricc_variant_min_side": (ctypes.c_int, [ctypes.c_int]),
    "tricc_graph_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    "tricc_graph_build": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, _P, _P, _P, ctypes.c_size_t,
                                         ctypes.POINTER(Tuning), _P, ctypes.POINTER(_P)]),
    "tricc_graph_from_csr": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, _P, _P, ctypes.c_int, _P,
                                            ctypes.c_size_t, ctypes.POINTER(Tuning), _P, ctypes.POINTER(_P)]),
    "tricc_graph_info_get": (ctypes.c_int, [_P, ctypes.POINTER(GraphInfo)]),
    "tricc_graph_retune": (ctypes.c_int, [_P, ctypes.POINTER(Tuning), _P]),
    "tricc_graph_stats": (ctypes.c_int, [_P, _P]),
    "tricc_count": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "tricc_graph_has_edges": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, _P, _P]),
    "tricc_core_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "tricc_graph_count_k4": (ctypes.c_int, [_P, _P, _P]),
    "tricc_graph_count_k5": (ctypes.c_int, [_P, _P, _P]),
    "tricc_graph_degeneracy": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int32), _P]),
    "tricc_graph_reorient": (ctypes.c_int, [_P, _P, _P]),
    "tricc_graph_core": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int32),
                                        _P]),
    "tricc_count_begin": (ctypes.c_int, [_P, _P, _P]),
    "tricc_count_bin": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "tricc_count_bins": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, _P]),
    "tricc_count_finish": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "tricc_count_check": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64), _P]),
    "tricc_probe_copy": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
    "tricc_gen_rmat": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64] + [ctypes.c_double] * 5
                       + [ctypes.c_uint64, _P, _P, _P, _P]),
    "tricc_gen_er_workspace_size": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    "tricc_gen_er": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, _P, _P, _P, ctypes.c_size_t, _P]),
    "tricc_gen_ba_edges": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_int32]),
    "tricc_gen_ba_workspace_size": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "tricc_gen_ba": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, _P, _P, _P, ctypes.c_size_t, _P]),
    "tricc_graph_arrays": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                          ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    "tricc_graph_free": (None, [_P]),
    "tricc_count_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, _P, _P, _P, _P, _P, _P, _P]),
    "tricc_batch_default_tuning": (ctypes.c_int, [ctypes.POINTER(BatchTuning)]),
    "tricc_batch_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                                  ctypes.POINTER(ctypes.c_size_t)]),
    "tricc_batch_build": (ctypes.c_int, [ctypes.c_int32, _P, _P, _P, _P, _P, ctypes.c_size_t,
                                         ctypes.POINTER(BatchTuning), _P, ctypes.POINTER(_P)]),
    "tricc_batch_build_csr": (ctypes.c_int, [ctypes.c_int32, _P, ctypes.c_int64, _P, _P, ctypes.c_int, _P,
                                             ctypes.c_size_t, ctypes.POINTER(BatchTuning), _P, ctypes.POINTER(_P)]),
    "tricc_batch_plan": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "tricc_batch_bind": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "tricc_batch_run": (ctypes.c_int, [_P, _P]),
    "tricc_batch_run_eager": (ctypes.c_int, [_P, _P]),
    "tricc_batch_retune": (ctypes.c_int, [_P, ctypes.POINTER(BatchTuning), _P]),
    "tricc_batch_info_get": (ctypes.c_int, [_P, ctypes.POINTER(BatchInfo)]),
    "tricc_batch_graph": (_P, [_P]),
    "tricc_batch_free": (None, [_P]),
    "tricc_server_create": (ctypes.c_int, [_P, _P, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(_P)]),
    "tricc_server_now": (ctypes.c_double, [_P]),
    "tricc_server_set_tuning": (ctypes.c_int, [_P, ctypes.POINTER(BatchTuning)]),
    "tricc_server_query_bytes": (ctypes.c_size_t, [_P, _P, ctypes.c_int64]),
    "tricc_server_submit": (ctypes.c_int, [_P, ctypes.c_uint64, _P, ctypes.c_int64, ctypes.c_double]),
    "tricc_server_poll": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "tricc_server_drain": (ctypes.c_int, [_P]),
    "tricc_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "tricc_server_last_error": (ctypes.c_char_p, []),
    "tricc_server_free": (None, [_P]),
}


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                              "or python -m paper_1606_07550_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def status_str(status):
    return lib().tricc_status_str(status).decode()


def last_error():
    return lib().tricc_last_error().decode()


def check(status, what):
    if status != TRICC_OK:
        raise TriccError(status, what)
