"""Python binding of libnlfem (include/nlfem.h): argument marshalling only.

Every step of assembly and solve runs in the HIP library; PyTorch provides
device memory and the stream.  Importing this module loads the in-tree
libnlfem.so and raises if it is missing -- there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnlfem.so")

NLFEM_OK = 0
NLFEM_E_INVALID_ARG = 1
NLFEM_E_MESH = 2
NLFEM_E_OOM = 3
NLFEM_E_DEVICE = 4
NLFEM_E_NOT_CONVERGED = 5
NLFEM_E_UNSUPPORTED = 6
NLFEM_FP64 = 0
NLFEM_FP32_LOCAL = 1
NLFEM_MAX_MC_SAMPLES = 2047  # sample sums stay exact 32/64-bit integers
# ball approximation strategies (nlfem_strategy)
STRATEGIES = {"fullcaps": 0, "nocaps": 1, "overlap": 2, "inside": 3, "barycenter": 4}
# where the cap samples are drawn (nlfem_cap_sampling)
CAP_SAMPLING = {"whole": 0, "outside_ui": 1}
# Monte Carlo keying (nlfem_keying): samples per (point, element) pair or per element
KEYING = {"pair": 0, "element": 1}


def keying_id(kk):
    if isinstance(kk, str):
        if kk not in KEYING:
            raise ValueError(f"unknown keying {kk!r}")
        return KEYING[kk]
    return int(kk)


def cap_sampling_id(cs):
    if isinstance(cs, str):
        if cs not in CAP_SAMPLING:
            raise ValueError(f"unknown cap sampling {cs!r}")
        return CAP_SAMPLING[cs]
    return int(cs)


def strategy_id(st):
    if isinstance(st, str):
        if st not in STRATEGIES:
            raise ValueError(f"unknown strategy {st!r}")
        return STRATEGIES[st]
    return int(st)

STATUS_NAMES = {0: "OK", 1: "E_INVALID_ARG", 2: "E_MESH", 3: "E_OOM", 4: "E_DEVICE",
                5: "E_NOT_CONVERGED", 6: "E_UNSUPPORTED"}


class nlfem_mesh(C.Structure):
    _fields_ = [("n_vertices", C.c_int64), ("n_tets", C.c_int64), ("coords", C.c_void_p),
                ("tets", C.c_void_p), ("vertex_free", C.c_void_p), ("tet_region", C.c_void_p),
                ("mem_kind", C.c_int32)]


class nlfem_params(C.Structure):
    _fields_ = [("delta", C.c_double), ("psi", C.c_double), ("mc_samples", C.c_int32),
                ("seed", C.c_uint64), ("precision", C.c_int32), ("outer_mask", C.c_void_p),
                ("strategy", C.c_int32), ("cap_sampling", C.c_int32), ("keying", C.c_int32)]


class nlfem_pair_record(C.Structure):
    _fields_ = [("q", C.c_int32), ("m", C.c_int32), ("cls", C.c_int32), ("pad", C.c_int32),
                ("S", C.c_double * 15)]


class nlfem_solve_params(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32)]


class nlfem_request_info(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("n_free", C.c_int64), ("nnz_ff", C.c_int64),
                ("nnz_fc", C.c_int64), ("pair_counts", C.c_int64 * 5), ("cg_iters", C.c_int32),
                ("attempts", C.c_int32), ("cg_rel_residual", C.c_double), ("queue_s", C.c_double),
                ("plan_s", C.c_double), ("assemble_s", C.c_double), ("solve_s", C.c_double),
                ("latency_s", C.c_double), ("est_bytes", C.c_size_t), ("peak_bytes", C.c_size_t)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["pair_counts"] = list(self.pair_counts)
        return d


class nlfem_server_counters(C.Structure):
    _fields_ = [("queued", C.c_int64), ("running", C.c_int64), ("done", C.c_int64), ("failed", C.c_int64),
                ("max_running", C.c_int32), ("n_slots", C.c_int32), ("pool_bytes", C.c_size_t),
                ("pool_used", C.c_size_t), ("pool_peak", C.c_size_t)]


EXPORTS = ["nlfem_create", "nlfem_destroy", "nlfem_last_error", "nlfem_memory_in_use", "nlfem_trim",
           "nlfem_rule_constants", "nlfem_plan_create", "nlfem_plan_info", "nlfem_assemble",
           "nlfem_assemble_exact_g", "nlfem_cg", "nlfem_plan_cg", "nlfem_cg_noalloc",
           "nlfem_plan_destroy", "nlfem_debug_pairs", "nlfem_plan_timings",
           "nlfem_batch_create", "nlfem_batch_info", "nlfem_batch_assemble", "nlfem_batch_system",
           "nlfem_batch_tuning", "nlfem_batch_set_launch", "nlfem_batch_destroy",
           "nlfem_server_create", "nlfem_server_submit", "nlfem_server_poll", "nlfem_server_wait",
           "nlfem_server_take", "nlfem_server_stats", "nlfem_server_last_error", "nlfem_server_destroy"]

_lib = None


def load():
    """Loads libnlfem.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with paper_2302_07499_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i64 = C.c_int64
    L.nlfem_create.argtypes = [C.POINTER(P), C.c_int, P, C.c_size_t]
    L.nlfem_destroy.argtypes = [P]
    L.nlfem_last_error.argtypes = [P]
    L.nlfem_last_error.restype = C.c_char_p
    L.nlfem_memory_in_use.argtypes = [P, C.POINTER(C.c_size_t)]
    L.nlfem_trim.argtypes = [P]
    L.nlfem_rule_constants.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.nlfem_rule_constants.restype = None
    L.nlfem_plan_create.argtypes = [P, C.POINTER(nlfem_mesh), C.POINTER(nlfem_params), C.POINTER(P)]
    L.nlfem_plan_info.argtypes = [P, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64),
                                  C.POINTER(C.c_size_t)]
    L.nlfem_assemble.argtypes = [P] * 11
    L.nlfem_assemble_exact_g.argtypes = [P, P, P, C.c_int32, P] + [P] * 8
    L.nlfem_cg.argtypes = [P, i64, P, P, P, P, P, C.c_double, C.c_int32, C.POINTER(C.c_int32),
                           C.POINTER(C.c_double)]
    L.nlfem_plan_cg.argtypes = [P, P, P, P, C.c_double, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    L.nlfem_cg_noalloc.argtypes = L.nlfem_cg.argtypes
    L.nlfem_plan_destroy.argtypes = [P]
    L.nlfem_debug_pairs.argtypes = [P, i64, i64, P, i64, C.POINTER(i64)]
    L.nlfem_plan_timings.argtypes = [P, C.POINTER(C.c_double)]
    L.nlfem_batch_create.argtypes = [P, C.c_int32, C.POINTER(nlfem_mesh), C.POINTER(nlfem_params), C.POINTER(P)]
    L.nlfem_batch_info.argtypes = [P, C.c_int32, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    L.nlfem_batch_assemble.argtypes = [P, C.POINTER(P), C.POINTER(P)]
    L.nlfem_batch_system.argtypes = [P, C.c_int32] + [C.POINTER(P)] * 8
    L.nlfem_batch_tuning.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
    L.nlfem_batch_set_launch.argtypes = [P, C.c_int32, C.c_int32]
    L.nlfem_batch_destroy.argtypes = [P]
    L.nlfem_server_create.argtypes = [C.c_int, C.c_int32, C.c_size_t, C.POINTER(P)]
    L.nlfem_server_submit.argtypes = [P, C.POINTER(nlfem_mesh), C.POINTER(nlfem_params), P, P,
                                      C.POINTER(nlfem_solve_params), C.POINTER(C.c_uint64)]
    L.nlfem_server_poll.argtypes = [P, C.c_uint64, C.POINTER(nlfem_request_info)]
    L.nlfem_server_wait.argtypes = [P, C.c_uint64, C.c_double, C.POINTER(nlfem_request_info)]
    L.nlfem_server_take.argtypes = [P, C.c_uint64, P, P]
    L.nlfem_server_stats.argtypes = [P, C.POINTER(nlfem_server_counters)]
    L.nlfem_server_last_error.argtypes = [P]
    L.nlfem_server_last_error.restype = C.c_char_p
    L.nlfem_server_destroy.argtypes = [P]
    for name in EXPORTS:
        if name not in ("nlfem_rule_constants", "nlfem_last_error", "nlfem_server_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


class NlfemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(st, ctx=None):
    if st != NLFEM_OK:
        msg = load().nlfem_last_error(ctx).decode() if ctx else ""
        raise NlfemError(st, msg)


def last_error(ctx) -> str:
    """Message of the last failed call on the context."""
    return load().nlfem_last_error(ctx).decode()


# ---- thin wrappers with the C names ------------------------------------------

def nlfem_create(device: int = 0, stream=None, hbm_budget_bytes: int = 0):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    h = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    ctx = C.c_void_p()
    _check(load().nlfem_create(C.byref(ctx), device, C.c_void_p(h), hbm_budget_bytes))
    return ctx


def nlfem_destroy(ctx):
    _check(load().nlfem_destroy(ctx))


def nlfem_last_error(ctx) -> str:
    return load().nlfem_last_error(ctx).decode()


def nlfem_memory_in_use(ctx) -> int:
    b = C.c_size_t()
    _check(load().nlfem_memory_in_use(ctx, C.byref(b)), ctx)
    return b.value


def nlfem_trim(ctx):
    _check(load().nlfem_trim(ctx), ctx)


def nlfem_rule_constants():
    a, b = C.c_double(), C.c_double()
    load().nlfem_rule_constants(C.byref(a), C.byref(b))
    return a.value, b.value


def nlfem_plan_create(ctx, mesh: nlfem_mesh, params: nlfem_params):
    plan = C.c_void_p()
    _check(load().nlfem_plan_create(ctx, C.byref(mesh), C.byref(params), C.byref(plan)), ctx)
    return plan


def nlfem_plan_info(plan):
    nf, nff, nfc = C.c_int64(), C.c_int64(), C.c_int64()
    pc = (C.c_int64 * 5)()
    ws = C.c_size_t()
    _check(load().nlfem_plan_info(plan, C.byref(nf), C.byref(nff), C.byref(nfc), pc, C.byref(ws)))
    return {"n_free": nf.value, "nnz_ff": nff.value, "nnz_fc": nfc.value, "pair_counts": list(pc),
            "workspace_bytes": ws.value}


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def nlfem_assemble(plan, f_qp, g_nodal, ff_row_ptr, ff_col, ff_val, fc_row_ptr, fc_col, fc_val, rhs,
                   free_to_vertex, ctx=None):
    st = load().nlfem_assemble(plan, _ptr(f_qp), _ptr(g_nodal), _ptr(ff_row_ptr), _ptr(ff_col), _ptr(ff_val),
                               _ptr(fc_row_ptr), _ptr(fc_col), _ptr(fc_val), _ptr(rhs), _ptr(free_to_vertex))
    _check(st, ctx)


def gpoly_coef(g_poly):
    """[a, b, c] array of the coefficients of y1^a y2^b y3^c -> (degree, flat
    float64 array with index a + n1 (b + n1 c), n1 = degree + 1)."""
    G = np.asarray(g_poly, dtype=np.float64)
    n1 = G.shape[0]
    if G.shape != (n1, n1, n1):
        raise ValueError("g_poly must be a cube array [a, b, c]")
    return n1 - 1, np.ascontiguousarray(G.transpose(2, 1, 0)).reshape(-1)


def nlfem_assemble_exact_g(plan, f_qp, g_nodal, g_poly, ff_row_ptr, ff_col, ff_val, fc_row_ptr, fc_col, fc_val,
                           rhs, free_to_vertex, ctx=None):
    deg, coef = gpoly_coef(g_poly)
    st = load().nlfem_assemble_exact_g(plan, _ptr(f_qp), _ptr(g_nodal), deg, coef.ctypes.data, _ptr(ff_row_ptr),
                                       _ptr(ff_col), _ptr(ff_val), _ptr(fc_row_ptr), _ptr(fc_col), _ptr(fc_val),
                                       _ptr(rhs), _ptr(free_to_vertex))
    _check(st, ctx)


def nlfem_cg(ctx, n, row_ptr, col, val, b, x, rtol=1e-10, max_iter=None):
    it, rr = C.c_int32(), C.c_double()
    st = load().nlfem_cg(ctx, n, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(b), _ptr(x), rtol,
                         n if max_iter is None else max_iter, C.byref(it), C.byref(rr))
    if st not in (NLFEM_OK, NLFEM_E_NOT_CONVERGED):
        _check(st, ctx)
    return it.value, rr.value, st == NLFEM_OK


def nlfem_cg_noalloc(ctx, n, row_ptr, col, val, b, x, rtol=1e-10, max_iter=None):
    """nlfem_cg with its work vectors in the library's static device scratch
    (no device allocation; n <= its maximum, else NlfemError)."""
    it, rr = C.c_int32(), C.c_double()
    st = load().nlfem_cg_noalloc(ctx, n, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(b), _ptr(x), rtol,
                                 n if max_iter is None else max_iter, C.byref(it), C.byref(rr))
    if st not in (NLFEM_OK, NLFEM_E_NOT_CONVERGED):
        _check(st, ctx)
    return it.value, rr.value, st == NLFEM_OK


def nlfem_plan_cg(plan, n_free, ff_val, rhs, x, rtol=1e-10, max_iter=None, ctx=None):
    """CG on the plan's own A_ff pattern with the caller's values."""
    it, rr = C.c_int32(), C.c_double()
    st = load().nlfem_plan_cg(plan, _ptr(ff_val), _ptr(rhs), _ptr(x), rtol,
                              n_free if max_iter is None else max_iter, C.byref(it), C.byref(rr))
    if st not in (NLFEM_OK, NLFEM_E_NOT_CONVERGED):
        _check(st, ctx)
    return it.value, rr.value, st == NLFEM_OK


def nlfem_plan_destroy(plan):
    _check(load().nlfem_plan_destroy(plan))


def nlfem_debug_pairs(plan, q_begin, q_end, ctx=None):
    n = C.c_int64()
    st = load().nlfem_debug_pairs(plan, q_begin, q_end, None, 0, C.byref(n))
    if st not in (NLFEM_OK, NLFEM_E_INVALID_ARG):
        _check(st, ctx)
    cnt = n.value
    buf = (nlfem_pair_record * max(cnt, 1))()
    _check(load().nlfem_debug_pairs(plan, q_begin, q_end, C.cast(buf, C.c_void_p), cnt, C.byref(n)), ctx)
    rec = np.ctypeslib.as_array(buf)[:cnt]
    return {"q": rec["q"].copy(), "m": rec["m"].copy(), "cls": rec["cls"].copy(), "S": rec["S"].copy()}


def nlfem_plan_timings(plan):
    t = (C.c_double * 6)()
    _check(load().nlfem_plan_timings(plan, t))
    return list(t)


# ---- convenience: one problem on the GPU -------------------------------------

@dataclass
class System:
    n_free: int
    ff_row_ptr: object
    ff_col: object
    ff_val: object
    fc_row_ptr: object
    fc_col: object
    fc_val: object
    rhs: object
    free_to_vertex: object
    info: dict


_OPEN_DEVICES = weakref.WeakSet()


class Device:
    """A context bound to a torch device and its current stream.  Plans made
    from it are destroyed before the context (close(), or at interpreter exit)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        import torch
        self.torch = torch
        self.device = device
        self.dev = torch.device("cuda", device)
        self.ctx = nlfem_create(device, torch.cuda.current_stream(device), hbm_budget_bytes)
        self.plans = weakref.WeakSet()
        _OPEN_DEVICES.add(self)

    def close(self):
        for p in list(self.plans):
            p.destroy()
        if self.ctx is not None:
            nlfem_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def to_dev(self, a, dtype):
        return self.torch.as_tensor(np.ascontiguousarray(a)).to(self.dev, dtype=dtype)

    def mesh(self, coords, tets, vertex_free, tet_region=None):
        t = self.torch
        keep = {"coords": self.to_dev(coords, t.float64), "tets": self.to_dev(tets, t.int32),
                "vfree": self.to_dev(vertex_free, t.uint8),
                "region": None if tet_region is None else self.to_dev(tet_region, t.uint8)}
        m = nlfem_mesh(int(keep["coords"].shape[0]), int(keep["tets"].shape[0]), keep["coords"].data_ptr(),
                       keep["tets"].data_ptr(), keep["vfree"].data_ptr(),
                       None if keep["region"] is None else keep["region"].data_ptr(), 1)
        return m, keep

    def plan(self, coords, tets, vertex_free, delta, psi, mc_samples, seed, precision="fp64", tet_region=None,
             outer_mask=None, strategy="fullcaps", cap_sampling="whole", keying="pair"):
        m, keep = self.mesh(coords, tets, vertex_free, tet_region)
        om = None if outer_mask is None else self.to_dev(outer_mask, self.torch.uint8)
        prm = nlfem_params(float(delta), float(psi), int(mc_samples), int(seed),
                           NLFEM_FP32_LOCAL if precision == "fp32" else NLFEM_FP64,
                           None if om is None else om.data_ptr(), strategy_id(strategy),
                           cap_sampling_id(cap_sampling), keying_id(keying))
        plan = nlfem_plan_create(self.ctx, m, prm)
        return Plan(self, plan)

    def plan_problem(self, pb, outer_mask=None):
        mm = pb.mesh
        return self.plan(mm.coords, mm.tets, pb.vertex_free, pb.delta, pb.psi, pb.mc_samples, pb.seed,
                         precision=pb.precision, outer_mask=outer_mask, tet_region=getattr(pb, "tet_region", None),
                         strategy=getattr(pb, "strategy", "fullcaps"),
                         cap_sampling=getattr(pb, "cap_sampling", "whole"),
                         keying=getattr(pb, "keying", "pair"))


class Plan:
    def __init__(self, dev: Device, handle):
        self.dev = dev
        self.handle = handle
        self.info = nlfem_plan_info(handle)
        dev.plans.add(self)

    def destroy(self):
        if self.handle is not None and self.dev.ctx is not None:
            nlfem_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def alloc_system(self) -> System:
        t = self.dev.torch
        d = self.dev.dev
        nf, nff, nfc = self.info["n_free"], self.info["nnz_ff"], self.info["nnz_fc"]
        return System(nf, t.empty(nf + 1, dtype=t.int64, device=d), t.empty(max(nff, 1), dtype=t.int32, device=d),
                      t.empty(max(nff, 1), dtype=t.float64, device=d), t.empty(nf + 1, dtype=t.int64, device=d),
                      t.empty(max(nfc, 1), dtype=t.int32, device=d), t.empty(max(nfc, 1), dtype=t.float64, device=d),
                      t.empty(max(nf, 1), dtype=t.float64, device=d), t.empty(max(nf, 1), dtype=t.int32, device=d),
                      dict(self.info))

    def assemble(self, f_qp=None, g_nodal=None, out: System | None = None, g_poly=None) -> System:
        """g_poly (tensor coefficients [a, b, c] of g): the paper-exact
        right-hand side (nlfem_assemble_exact_g); else nodal g only."""
        t = self.dev.torch
        sysm = out if out is not None else self.alloc_system()
        fq = None if f_qp is None else (f_qp if isinstance(f_qp, t.Tensor) else self.dev.to_dev(f_qp, t.float64))
        gn = None if g_nodal is None else (g_nodal if isinstance(g_nodal, t.Tensor)
                                           else self.dev.to_dev(g_nodal, t.float64))
        if g_poly is None:
            nlfem_assemble(self.handle, fq, gn, sysm.ff_row_ptr, sysm.ff_col, sysm.ff_val, sysm.fc_row_ptr,
                           sysm.fc_col, sysm.fc_val, sysm.rhs, sysm.free_to_vertex, ctx=self.dev.ctx)
        else:
            nlfem_assemble_exact_g(self.handle, fq, gn, g_poly, sysm.ff_row_ptr, sysm.ff_col, sysm.ff_val,
                                   sysm.fc_row_ptr, sysm.fc_col, sysm.fc_val, sysm.rhs, sysm.free_to_vertex,
                                   ctx=self.dev.ctx)
        sysm._keep = (fq, gn)
        return sysm

    def solve(self, sysm: System, rtol=1e-10, max_iter=None):
        t = self.dev.torch
        x = t.zeros(max(sysm.n_free, 1), dtype=t.float64, device=self.dev.dev)
        it, rr, ok = nlfem_cg(self.dev.ctx, sysm.n_free, sysm.ff_row_ptr, sysm.ff_col, sysm.ff_val, sysm.rhs, x,
                              rtol, max_iter)
        return x[:sysm.n_free], it, rr, ok

    def timings(self):
        return nlfem_plan_timings(self.handle)

    def debug_pairs(self, q_begin, q_end):
        return nlfem_debug_pairs(self.handle, q_begin, q_end, ctx=self.dev.ctx)


class Batch:
    """Many meshes assembled by one persistent fused launch replayed from a HIP graph."""

    def __init__(self, dev: Device, problems, outer_masks=None):
        t = dev.torch
        self.dev = dev
        self.n = len(problems)
        self.keep = []
        meshes = (nlfem_mesh * max(self.n, 1))()
        params = (nlfem_params * max(self.n, 1))()
        for i, pb in enumerate(problems):
            m, keep = dev.mesh(pb.mesh.coords, pb.mesh.tets, pb.vertex_free, getattr(pb, "tet_region", None))
            om = None
            if outer_masks is not None and outer_masks[i] is not None:
                om = dev.to_dev(outer_masks[i], t.uint8)
            self.keep.append((keep, om))
            meshes[i] = m
            params[i] = nlfem_params(float(pb.delta), float(pb.psi), int(pb.mc_samples), int(pb.seed),
                                     NLFEM_FP32_LOCAL if pb.precision == "fp32" else NLFEM_FP64,
                                     None if om is None else om.data_ptr(),
                                     strategy_id(getattr(pb, "strategy", "fullcaps")),
                                     cap_sampling_id(getattr(pb, "cap_sampling", "whole")),
                                     keying_id(getattr(pb, "keying", "pair")))
        h = C.c_void_p()
        _check(load().nlfem_batch_create(dev.ctx, self.n, meshes, params, C.byref(h)), dev.ctx)
        self.handle = h
        self.infos = []
        for i in range(self.n):
            nf, nff, nfc = C.c_int64(), C.c_int64(), C.c_int64()
            pc = (C.c_int64 * 5)()
            _check(load().nlfem_batch_info(h, i, C.byref(nf), C.byref(nff), C.byref(nfc), pc))
            self.infos.append({"n_free": nf.value, "nnz_ff": nff.value, "nnz_fc": nfc.value, "pair_counts": list(pc)})
        self.inputs = None
        dev.plans.add(self)

    def set_inputs(self, f_list, g_list):
        t = self.dev.torch
        self.inputs = ([None if f is None else self.dev.to_dev(f, t.float64) for f in f_list],
                       [None if g is None else self.dev.to_dev(g, t.float64) for g in g_list])

    def assemble(self):
        fl, gl = self.inputs if self.inputs is not None else ([None] * self.n, [None] * self.n)
        fa = (C.c_void_p * max(self.n, 1))(*[None if f is None else f.data_ptr() for f in fl])
        ga = (C.c_void_p * max(self.n, 1))(*[None if g is None else g.data_ptr() for g in gl])
        _check(load().nlfem_batch_assemble(self.handle, fa, ga), self.dev.ctx)

    def system_numpy(self, i):
        import torch
        ptrs = [C.c_void_p() for _ in range(8)]
        _check(load().nlfem_batch_system(self.handle, i, *[C.byref(p) for p in ptrs]))
        info = self.infos[i]
        nf, nff, nfc = info["n_free"], info["nnz_ff"], info["nnz_fc"]
        sizes = [(nf + 1, np.int64), (nff, np.int32), (nff, np.float64), (nf + 1, np.int64), (nfc, np.int32),
                 (nfc, np.float64), (nf, np.float64), (nf, np.int32)]
        torch.cuda.synchronize()
        out = []
        for p, (cnt, dt) in zip(ptrs, sizes):
            a = np.empty(cnt, dtype=dt)
            if cnt:
                _hip_d2h(a, p.value)
            out.append(a)
        names = ["ff_row_ptr", "ff_col", "ff_val", "fc_row_ptr", "fc_col", "fc_val", "rhs", "free_to_vertex"]
        d = dict(zip(names, out))
        d["n_free"] = nf
        d["pair_counts"] = np.array(info["pair_counts"], dtype=np.int64)
        return d

    def tuning(self):
        b, g, tm, lm = C.c_int32(), C.c_int32(), C.c_double(), C.c_double()
        _check(load().nlfem_batch_tuning(self.handle, C.byref(b), C.byref(g), C.byref(tm), C.byref(lm)))
        return {"block": b.value, "grid": g.value, "tuned_integrate_ms": tm.value, "last_graph_ms": lm.value}

    def set_launch(self, block: int, wg_per_cu: int):
        """Pins every group's launch shape (wg_per_cu 0: one workgroup per item)."""
        _check(load().nlfem_batch_set_launch(self.handle, int(block), int(wg_per_cu)), self.dev.ctx)

    def destroy(self):
        if self.handle is not None and self.dev.ctx is not None:
            _check(load().nlfem_batch_destroy(self.handle))
        self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Server:
    """Request loop (include/nlfem.h, serving): submit problems, wait for
    their solutions; the library runs each request on one of its slots."""

    def __init__(self, device: int = 0, n_slots: int = 4, pool_bytes: int = 0):
        h = C.c_void_p()
        st = load().nlfem_server_create(device, n_slots, pool_bytes, C.byref(h))
        if st != NLFEM_OK:
            raise NlfemError(st, "nlfem_server_create failed")
        self.handle = h
        _OPEN_SERVERS.add(self)

    def _err(self, st):
        if st != NLFEM_OK:
            raise NlfemError(st, load().nlfem_server_last_error(self.handle).decode())

    def submit(self, pb, rtol: float = 1e-10, max_iter: int = 0, outer_mask=None) -> int:
        mesh = pb.mesh
        coords = np.ascontiguousarray(mesh.coords, dtype=np.float64)
        tets = np.ascontiguousarray(mesh.tets, dtype=np.int32)
        vfree = np.ascontiguousarray(pb.vertex_free, dtype=np.uint8)
        f = None if pb.f_qp is None else np.ascontiguousarray(pb.f_qp, dtype=np.float64)
        g = None if pb.g_nodal is None else np.ascontiguousarray(pb.g_nodal, dtype=np.float64)
        om = None if outer_mask is None else np.ascontiguousarray(outer_mask, dtype=np.uint8)
        tr = getattr(pb, "tet_region", None)
        tr = None if tr is None else np.ascontiguousarray(tr, dtype=np.uint8)
        m = nlfem_mesh(mesh.n_vertices, mesh.n_tets, coords.ctypes.data, tets.ctypes.data, vfree.ctypes.data,
                       None if tr is None else tr.ctypes.data, 0)
        prm = nlfem_params(float(pb.delta), float(pb.psi), int(pb.mc_samples), int(pb.seed),
                           NLFEM_FP32_LOCAL if pb.precision == "fp32" else NLFEM_FP64,
                           None if om is None else om.ctypes.data, strategy_id(getattr(pb, "strategy", "fullcaps")),
                           cap_sampling_id(getattr(pb, "cap_sampling", "whole")),
                           keying_id(getattr(pb, "keying", "pair")))
        sp = nlfem_solve_params(rtol, max_iter)
        t = C.c_uint64()
        self._err(load().nlfem_server_submit(self.handle, C.byref(m), C.byref(prm),
                                             None if f is None else f.ctypes.data,
                                             None if g is None else g.ctypes.data, C.byref(sp), C.byref(t)))
        return t.value

    def poll(self, ticket: int) -> dict:
        info = nlfem_request_info()
        self._err(load().nlfem_server_poll(self.handle, ticket, C.byref(info)))
        return info.as_dict()

    def wait(self, ticket: int, timeout: float = -1.0) -> dict:
        info = nlfem_request_info()
        self._err(load().nlfem_server_wait(self.handle, ticket, timeout, C.byref(info)))
        return info.as_dict()

    def take(self, ticket: int):
        """Solution x [n_free] and free_to_vertex [n_free] of a finished request."""
        info = self.poll(ticket)
        nf = int(info["n_free"])
        x = np.empty(nf, dtype=np.float64)
        f2v = np.empty(nf, dtype=np.int32)
        self._err(load().nlfem_server_take(self.handle, ticket, x.ctypes.data, f2v.ctypes.data))
        return x, f2v, info

    def stats(self) -> dict:
        c = nlfem_server_counters()
        self._err(load().nlfem_server_stats(self.handle, C.byref(c)))
        return {k: getattr(c, k) for k, _ in c._fields_}

    def close(self):
        if self.handle is not None:
            load().nlfem_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_OPEN_SERVERS = weakref.WeakSet()

_hip = None


def _hip_d2h(arr, dev_ptr):
    """Copies device memory owned by the library into a numpy array (hipMemcpy)."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    rc = _hip.hipMemcpy(arr.ctypes.data, C.c_void_p(dev_ptr), arr.nbytes, 2)  # hipMemcpyDeviceToHost
    if rc != 0:
        raise NlfemError(NLFEM_E_DEVICE, f"hipMemcpy failed ({rc})")


@atexit.register
def _close_all():
    for sv in list(_OPEN_SERVERS):
        try:
            sv.close()
        except Exception:
            pass
    for d in list(_OPEN_DEVICES):
        try:
            d.close()
        except Exception:
            pass


def system_to_numpy(s: System) -> dict:
    nf = s.n_free
    nff, nfc = s.info["nnz_ff"], s.info["nnz_fc"]
    return {"n_free": nf, "ff_row_ptr": s.ff_row_ptr.cpu().numpy(), "ff_col": s.ff_col[:nff].cpu().numpy(),
            "ff_val": s.ff_val[:nff].cpu().numpy(), "fc_row_ptr": s.fc_row_ptr.cpu().numpy(),
            "fc_col": s.fc_col[:nfc].cpu().numpy(), "fc_val": s.fc_val[:nfc].cpu().numpy(),
            "rhs": s.rhs[:nf].cpu().numpy(), "free_to_vertex": s.free_to_vertex[:nf].cpu().numpy(),
            "pair_counts": np.array(s.info["pair_counts"], dtype=np.int64)}
