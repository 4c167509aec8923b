"""Thin ctypes binding of libhlevy.so (include/hlevy.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Vectors are torch tensors on the GPU (float64, contiguous); streams default
to torch's current stream.  Importing this module fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhlevy.so")

HLEVY_OK = 0
PREC_FP64 = 0
PREC_MIXED = 1
PREC_MIXED_BF16 = 2
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "OOM", -3: "DEVICE", -4: "NOT_CONVERGED",
          -5: "RANK_CAP", -6: "BAD_HANDLE", -7: "ZERO_PIVOT"}


class Problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32), ("lo", C.c_double), ("hi", C.c_double),
                ("a", C.c_double), ("b", C.c_double * 2), ("c", C.c_double), ("s", C.c_double),
                ("lam", C.c_double), ("C", C.c_double), ("r0", C.c_double), ("kernel", C.c_int32),
                ("pad", C.c_int32), ("eps2", C.c_double), ("lam_neg", C.c_double),
                ("mask", C.POINTER(C.c_uint8)), ("s_field", C.POINTER(C.c_double))]


class HParams(C.Structure):
    _fields_ = [("leaf", C.c_int32), ("eta", C.c_double), ("n_block", C.c_int32),
                ("aca_tol", C.c_double), ("max_rank", C.c_int32), ("gather_waves", C.c_int32),
                ("rank_bucket", C.c_int32), ("strict_rank_cap", C.c_int32), ("taylor_rank", C.c_int32),
                ("cluster", C.c_int32)]


class Refine(C.Structure):
    _fields_ = [("tol", C.c_double), ("sweeps", C.c_int32), ("check_every", C.c_int32),
                ("max_sweeps", C.c_int32), ("pad", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("steps_done", C.c_int64), ("last_rel_residual", C.c_double), ("max_rel_residual", C.c_double),
                ("checks", C.c_int32), ("max_sweeps_used", C.c_int32), ("rank_overflows", C.c_int32),
                ("pad", C.c_int32), ("seconds", C.c_double)]


class Allocator(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)), ("ctx", C.c_void_p)]


class PlanInfo(C.Structure):
    _fields_ = [("N", C.c_int64), ("depth", C.c_int32), ("n_clusters", C.c_int32),
                ("n_dense", C.c_int32), ("n_lowrank", C.c_int32), ("max_leaf_points", C.c_int32),
                ("min_leaf_points", C.c_int32), ("dense_entries", C.c_int64)]


class OpInfo(C.Structure):
    _fields_ = [("dense_entries", C.c_int64), ("lowrank_entries", C.c_int64), ("max_rank", C.c_int32),
                ("mean_rank", C.c_double), ("rank_overflows", C.c_int32), ("subdivided_blocks", C.c_int32),
                ("device_bytes", C.c_size_t)]


class FacInfo(C.Structure):
    _fields_ = [("device_bytes", C.c_size_t), ("rank_overflows", C.c_int32), ("max_rank", C.c_int32),
                ("product_bytes", C.c_double * 3), ("lu_tol", C.c_double), ("dt", C.c_double),
                ("prec", C.c_int32), ("pad", C.c_int32)]


class KernelTimes(C.Structure):
    _fields_ = [("N", C.c_int64), ("reps", C.c_int32), ("pad", C.c_int32),
                ("project_ms", C.c_double * 3), ("gather_ms", C.c_double * 3),
                ("dense_bytes", C.c_double * 3), ("u_bytes", C.c_double * 3),
                ("v_bytes", C.c_double * 3), ("partial_bytes", C.c_double * 3)]


class TuneResult(C.Structure):
    _fields_ = [("leaf", C.c_int32), ("gather_waves", C.c_int32), ("rank_bucket", C.c_int32),
                ("from_cache", C.c_int32), ("ncand", C.c_int32), ("pad", C.c_int32),
                ("seconds", C.c_double), ("default_seconds", C.c_double),
                ("cand_leaf", C.c_int32 * 16), ("cand_gather_waves", C.c_int32 * 16),
                ("cand_rank_bucket", C.c_int32 * 16), ("cand_seconds", C.c_double * 16)]


EXPORTS = ["hlevy_abi_version", "hlevy_autotune", "hlevy_last_error", "hlevy_plan_info", "hlevy_footprint", "hlevy_assemble",
           "hlevy_assemble_batched", "hlevy_op_constants", "hlevy_exterior_forcing", "hlevy_exterior_forcing_far", "hlevy_op_info", "hlevy_fac_info", "hlevy_matvec",
           "hlevy_op_densify", "hlevy_factor", "hlevy_factor_batched", "hlevy_solve", "hlevy_solve_noalloc", "hlevy_krylov_solve", "hlevy_step",
           "hlevy_step_batched", "hlevy_fac_kernel_times", "hlevy_fac_apply", "hlevy_op_destroy", "hlevy_fac_destroy",
           "hlevy_server_create", "hlevy_server_submit", "hlevy_server_poll", "hlevy_server_take_failed",
           "hlevy_server_stats_get", "hlevy_server_destroy"]


KRYLOV_CG, KRYLOV_BICGSTAB, KRYLOV_GMRES = 0, 1, 2


class KrylovOpts(C.Structure):
    _fields_ = [("method", C.c_int32), ("max_iter", C.c_int32), ("tol", C.c_double), ("shift", C.c_double),
                ("precondition", C.c_int32), ("use_guess", C.c_int32), ("op", C.c_void_p),
                ("restart", C.c_int32), ("pad", C.c_int32)]


class KrylovStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("rel_residual", C.c_double),
                ("seconds", C.c_double)]


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("prec", C.c_int32), ("lu_tol", C.c_double), ("sweeps", C.c_int32),
                ("chunk", C.c_int32), ("max_active", C.c_int32), ("tol", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("active", C.c_int64), ("queued", C.c_int64),
                ("cache_hits", C.c_int64), ("cache_misses", C.c_int64), ("evictions", C.c_int64),
                ("cached_operators", C.c_int64), ("problem_steps", C.c_int64), ("bytes_in_use", C.c_size_t),
                ("assemble_seconds", C.c_double), ("factor_seconds", C.c_double), ("step_seconds", C.c_double),
                ("failed", C.c_int64), ("not_converged", C.c_int64), ("max_rel_residual", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhlevy.so is not built: run `python -m paper_1812_08324_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, st = C.c_void_p, C.c_int
    sig = {
        "hlevy_abi_version": ([], C.c_int32),
        "hlevy_last_error": ([], C.c_char_p),
        "hlevy_plan_info": ([C.POINTER(Problem), C.POINTER(HParams), C.POINTER(PlanInfo)], st),
        "hlevy_footprint": ([C.POINTER(Problem), C.POINTER(HParams), C.c_int32, C.POINTER(C.c_size_t)], st),
        "hlevy_assemble": ([C.POINTER(Problem), C.POINTER(HParams), C.POINTER(Allocator), vp, C.POINTER(vp)], st),
        "hlevy_assemble_batched": ([C.POINTER(Problem), C.POINTER(HParams), C.c_int32, C.POINTER(Allocator), vp,
                                    C.POINTER(vp)], st),
        "hlevy_op_constants": ([vp, C.POINTER(C.c_double), vp], st),
        "hlevy_op_info": ([vp, C.POINTER(OpInfo), vp], st),
        "hlevy_exterior_forcing": ([vp, vp, vp, vp], st),
        "hlevy_exterior_forcing_far": ([vp, vp, C.c_int32, C.c_double, C.c_double, vp, vp], st),
        "hlevy_fac_info": ([vp, C.POINTER(FacInfo), vp], st),
        "hlevy_matvec": ([vp, vp, vp, vp], st),
        "hlevy_op_densify": ([vp, vp, vp], st),
        "hlevy_factor": ([vp, C.c_double, C.c_int32, C.c_double, vp, C.POINTER(vp)], st),
        "hlevy_factor_batched": ([C.POINTER(vp), C.POINTER(C.c_double), C.c_int32, C.c_int32, C.c_double,
                                  C.c_size_t, vp, C.POINTER(vp)], st),
        "hlevy_solve": ([vp, vp, vp, C.c_int64, C.c_int64, C.POINTER(Refine), C.POINTER(Stats), vp], st),
        "hlevy_solve_noalloc": ([vp, vp, vp, C.POINTER(Refine), C.POINTER(Stats), vp], st),
        "hlevy_krylov_solve": ([vp, vp, vp, C.POINTER(KrylovOpts), C.POINTER(KrylovStats), C.POINTER(C.c_double),
                                vp], st),
        "hlevy_step_batched": ([C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_int64), C.c_int32, C.POINTER(Refine),
                                C.POINTER(Stats), vp], st),
        "hlevy_step": ([vp, vp, C.c_int64, vp, C.POINTER(C.c_double), C.POINTER(Refine),
                        C.POINTER(Stats), vp], st),
        "hlevy_fac_kernel_times": ([vp, C.c_int32, vp, C.POINTER(KernelTimes)], st),
        "hlevy_fac_apply": ([vp, C.c_int32, vp, vp, vp], st),
        "hlevy_autotune": ([C.POINTER(Problem), C.POINTER(HParams), C.c_double, C.c_int32, C.c_double, C.c_int64,
                            C.c_int32, C.c_char_p, vp, C.POINTER(TuneResult)], st),
        "hlevy_server_create": ([C.POINTER(ServerConfig), vp, C.POINTER(vp)], st),
        "hlevy_server_submit": ([vp, C.POINTER(Problem), C.POINTER(HParams), C.c_double, C.c_int64, vp, vp,
                                 C.POINTER(C.c_int64)], st),
        "hlevy_server_poll": ([vp, C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32)], st),
        "hlevy_server_take_failed": ([vp, C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32)], st),
        "hlevy_server_stats_get": ([vp, C.POINTER(ServerStats)], st),
        "hlevy_server_destroy": ([vp], None),
        "hlevy_op_destroy": ([vp], None),
        "hlevy_fac_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


class HlevyError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib.hlevy_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(status: int, where: str):
    if status != HLEVY_OK:
        raise HlevyError(status, where)


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dptr(t, n=None):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


KERNEL_TEMPERED, KERNEL_GAUSSIAN, KERNEL_TEMPERED_ASYM, KERNEL_VARIABLE_ORDER = 0, 1, 2, 3
CLUSTER_BISECT, CLUSTER_KMEANS = 0, 1


def make_problem(dim, n, lo, hi, s, lam=0.0, C_=None, a=0.0, b=(0.0, 0.0), c=0.0, r0=0.2, kernel=0,
                 eps2=0.0, lam_neg=None, mask=None, s_field=None) -> Problem:
    """lam_neg: the tempering rate of the jumps y < 0 (2D: y_1 < 0, the kernel
    tilted along the first axis); given, the kernel is
    HLEVY_KERNEL_TEMPERED_ASYM with lam for y > 0.  mask (2D): n x n
    array, nonzero = grid point in the domain.  s_field: one jump index per
    unknown (natural order); given, the kernel is HLEVY_KERNEL_VARIABLE_ORDER.
    The problem keeps its own copies of both arrays."""
    p = Problem()
    p.dim, p.n, p.lo, p.hi = int(dim), int(n), float(lo), float(hi)
    p.a, p.c, p.s, p.lam = float(a), float(c), float(s), float(lam)
    p.b[0], p.b[1] = float(b[0]), float(b[1] if len(b) > 1 else 0.0)
    p.C = -1.0 if C_ is None else float(C_)
    p.r0 = float(r0)
    p.kernel, p.eps2 = int(kernel), float(eps2)
    if lam_neg is not None:
        p.kernel, p.lam_neg = KERNEL_TEMPERED_ASYM, float(lam_neg)
    if mask is not None:
        m = (C.c_uint8 * (int(n) * int(n)))(*[1 if v else 0 for v in _flat(mask)])
        p._mask_arr, p._N = m, sum(m)
        p.mask = C.cast(m, C.POINTER(C.c_uint8))
    if s_field is not None:
        vals = [float(v) for v in _flat(s_field)]
        f = (C.c_double * len(vals))(*vals)
        p._s_arr = f
        p.s_field = C.cast(f, C.POINTER(C.c_double))
        p.kernel = KERNEL_VARIABLE_ORDER
    return p


def _flat(a):
    return a.reshape(-1).tolist() if hasattr(a, "reshape") else list(a)


def problem_N(prob: Problem) -> int:
    """Unknowns of a problem: n^dim, or the points its mask keeps."""
    n = getattr(prob, "_N", None)
    if n is not None:
        return int(n)
    return prob.n if prob.dim == 1 else prob.n * prob.n


def make_hparams(leaf=64, eta=1.0, n_block=4, aca_tol=1e-10, max_rank=16, gather_waves=0, rank_bucket=0,
                 strict_rank_cap=0, taylor_rank=0, cluster=CLUSTER_BISECT) -> HParams:
    h = HParams()
    h.leaf, h.eta, h.n_block, h.aca_tol, h.max_rank = int(leaf), float(eta), int(n_block), float(aca_tol), int(max_rank)
    h.gather_waves, h.rank_bucket, h.strict_rank_cap = int(gather_waves), int(rank_bucket), int(strict_rank_cap)
    h.taylor_rank, h.cluster = int(taylor_rank), int(cluster)
    return h


def footprint(prob: Problem, hp: HParams, prec: int = PREC_FP64) -> int:
    """Resident device bytes of an operator plus one factor (hlevy_footprint)."""
    out = C.c_size_t()
    _check(lib.hlevy_footprint(C.byref(prob), C.byref(hp), int(prec), C.byref(out)), "hlevy_footprint")
    return out.value


class TorchAllocator:
    """hlevy_allocator backed by torch's caching allocator: the library's
    device memory then shows in torch.cuda.memory_allocated().  Keep the
    object alive as long as the handles that used it."""

    def __init__(self, device=None):
        import torch
        self._torch = torch
        self.device = torch.cuda.current_device() if device is None else int(device)
        self._a = Allocator._fields_[0][1](self._alloc)
        self._f = Allocator._fields_[1][1](self._free)
        self.c = Allocator(self._a, self._f, None)

    def _alloc(self, nbytes, ctx):
        try:
            return self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device)
        except RuntimeError:
            return None

    def _free(self, p, ctx):
        self._torch.cuda.caching_allocator_delete(p)


def autotune(prob: Problem, hp: HParams, dt: float, prec: int, lu_tol: float, nsteps: int, batch: int = 1,
             cache=None, stream=None):
    """hlevy_autotune: returns (HParams with the chosen leaf and tile shapes,
    the result as a dict).  With a cache file whose key matches, no device
    work runs (and no stream is needed)."""
    out = TuneResult()
    path = None if cache is None else os.fsencode(cache)
    _check(lib.hlevy_autotune(C.byref(prob), C.byref(hp), float(dt), int(prec), float(lu_tol), int(nsteps),
                              int(batch), path, _stream(stream), C.byref(out)), "hlevy_autotune")
    n = out.ncand
    res = {"leaf": out.leaf, "gather_waves": out.gather_waves, "rank_bucket": out.rank_bucket,
           "from_cache": bool(out.from_cache), "seconds": out.seconds, "default_seconds": out.default_seconds,
           "candidates": [{"leaf": out.cand_leaf[i], "gather_waves": out.cand_gather_waves[i],
                           "rank_bucket": out.cand_rank_bucket[i], "seconds": out.cand_seconds[i]}
                          for i in range(n)]}
    tuned = HParams.from_buffer_copy(hp)
    tuned.leaf, tuned.gather_waves, tuned.rank_bucket = out.leaf, out.gather_waves, out.rank_bucket
    return tuned, res


def plan_info(prob: Problem, hp: HParams) -> dict:
    out = PlanInfo()
    _check(lib.hlevy_plan_info(C.byref(prob), C.byref(hp), C.byref(out)), "hlevy_plan_info")
    return {k: getattr(out, k) for k, _ in PlanInfo._fields_}


def fac_kernel_times(fac, reps: int = 20, stream=None) -> dict:
    """HIP-event timing of the per-step products in stepping order; returns
    {"G"|"Linv"|"Uinv": {project_ms, gather_ms, dense_bytes, u_bytes, v_bytes,
    partial_bytes}, "N": N}."""
    out = KernelTimes()
    _check(lib.hlevy_fac_kernel_times(fac.h, int(reps), _stream(stream), C.byref(out)), "hlevy_fac_kernel_times")
    res = {"N": out.N}
    for w, name in enumerate(("G", "Linv", "Uinv")):
        res[name] = {k: getattr(out, k)[w] for k in ("project_ms", "gather_ms", "dense_bytes", "u_bytes",
                                                      "v_bytes", "partial_bytes")}
    return res


class Op:
    """Assembled H-matrix of the generator G (handle owner)."""

    def __init__(self, prob: Problem, hp: HParams, stream=None, handle=None, allocator=None):
        if handle is None:
            handle = C.c_void_p()
            al = C.byref(allocator.c) if allocator is not None else None
            _check(lib.hlevy_assemble(C.byref(prob), C.byref(hp), al, _stream(stream), C.byref(handle)),
                   "hlevy_assemble")
        self.allocator = allocator   # must outlive the handle
        self.h = handle
        self.N = problem_N(prob)
        self.prob, self.hp = prob, hp

    def __del__(self):
        if getattr(self, "h", None) and self.h.value and lib is not None:
            lib.hlevy_op_destroy(self.h)
            self.h = None


class Fac:
    """H-LU factors of I - dt/2 G with their inverses (handle owner)."""

    def __init__(self, op: Op, dt: float, prec: int = PREC_FP64, lu_tol: float = 1e-12, stream=None,
                 handle=None):
        if handle is None:
            handle = C.c_void_p()
            _check(lib.hlevy_factor(op.h, float(dt), int(prec), float(lu_tol), _stream(stream),
                                    C.byref(handle)), "hlevy_factor")
        self.h = handle
        self.op = op           # the factor references the operator
        self.N = op.N
        self.dt = float(dt)

    def __del__(self):
        if getattr(self, "h", None) and self.h.value and lib is not None:
            lib.hlevy_fac_destroy(self.h)
            self.h = None


def assemble(prob: Problem, hp: HParams, stream=None, allocator=None) -> Op:
    return Op(prob, hp, stream, allocator=allocator)


def assemble_batched(probs, hps, stream=None) -> list:
    """Operators of several problems from one batched assembly
    (hlevy_assemble_batched)."""
    n = len(probs)
    if len(hps) != n or n == 0:
        raise ValueError("one hparams per problem, at least one problem")
    pa = (Problem * n)(*probs)
    ha = (HParams * n)(*hps)
    out = (C.c_void_p * n)()
    _check(lib.hlevy_assemble_batched(pa, ha, n, None, _stream(stream), out), "hlevy_assemble_batched")
    return [Op(p, hp, handle=C.c_void_p(out[i])) for i, (p, hp) in enumerate(zip(probs, hps))]


def op_constants(op: Op, stream=None):
    """[S0, S2, C2, T, S1]."""
    out = (C.c_double * 5)()
    _check(lib.hlevy_op_constants(op.h, out, _stream(stream)), "hlevy_op_constants")
    return list(out)


def exterior_forcing(op: Op, u_ext, g, stream=None):
    """g = the forcing of the exterior values u_ext (hlevy_exterior_forcing;
    1D: u_ext holds 2 (n + 1) values; 2D: (3 n + 2)^2 values on the extended
    lattice, interior entries ignored; g holds N values; float64 CUDA)."""
    n = op.prob.n
    ne = 2 * (n + 1) if op.prob.dim == 1 else (3 * n + 2) ** 2
    _check(lib.hlevy_exterior_forcing(op.h, _dptr(u_ext, ne), _dptr(g, op.N), _stream(stream)),
           "hlevy_exterior_forcing")


def exterior_forcing_far(op: Op, u_ext, next_: int, tail_left: float, tail_right: float, g, stream=None):
    """g = the exterior forcing with the far field f^{L_W}
    (hlevy_exterior_forcing_far; 1D: u_ext holds next_ values left of the
    box and next_ right of it; 2D: the extended lattice of
    (n + 2 next_)^2 values; beyond it the constant tails)."""
    n = op.N
    m = 2 * int(next_) if op.prob.dim == 1 else (op.prob.n + 2 * int(next_)) ** 2
    _check(lib.hlevy_exterior_forcing_far(op.h, _dptr(u_ext, m), int(next_), float(tail_left),
                                          float(tail_right), _dptr(g, n), _stream(stream)),
           "hlevy_exterior_forcing_far")


def op_info(op: Op, stream=None) -> dict:
    out = OpInfo()
    _check(lib.hlevy_op_info(op.h, C.byref(out), _stream(stream)), "hlevy_op_info")
    return {k: getattr(out, k) for k, _ in OpInfo._fields_}


def fac_info(fac, stream=None) -> dict:
    out = FacInfo()
    _check(lib.hlevy_fac_info(fac.h, C.byref(out), _stream(stream)), "hlevy_fac_info")
    d = {k: getattr(out, k) for k, _ in FacInfo._fields_}
    d["product_bytes"] = list(out.product_bytes)
    return d


def matvec(op: Op, x, y, stream=None):
    _check(lib.hlevy_matvec(op.h, _dptr(x, op.N), _dptr(y, op.N), _stream(stream)), "hlevy_matvec")


def op_densify(op: Op, dense, stream=None):
    _check(lib.hlevy_op_densify(op.h, _dptr(dense, op.N * op.N), _stream(stream)), "hlevy_op_densify")


def factor(op: Op, dt: float, prec: int = PREC_FP64, lu_tol: float = 1e-12, stream=None) -> Fac:
    return Fac(op, dt, prec, lu_tol, stream)


def factor_batched(ops, dts, prec: int = PREC_FP64, lu_tol: float = 1e-12, workspace_bytes: int = 0,
                   stream=None) -> list:
    """Factors of several problems from one joint plan (hlevy_factor_batched)."""
    n = len(ops)
    if len(dts) != n or n == 0:
        raise ValueError("one dt per operator, at least one operator")
    hs = (C.c_void_p * n)(*[o.h.value for o in ops])
    dv = (C.c_double * n)(*[float(d) for d in dts])
    out = (C.c_void_p * n)()
    _check(lib.hlevy_factor_batched(hs, dv, n, int(prec), float(lu_tol), int(workspace_bytes), _stream(stream),
                                    out), "hlevy_factor_batched")
    return [Fac(o, d, prec, lu_tol, handle=C.c_void_p(out[i])) for i, (o, d) in enumerate(zip(ops, dts))]


def _stats_dict(st):
    return {k: getattr(st, k) for k, _ in Stats._fields_ if k != "pad"}


def step_batched(facs, us, nsteps, refine=None, stats=False, stream=None):
    """Unforced Crank-Nicolson steps of every problem (hlevy_step_batched);
    nsteps: one count for all, or one per problem."""
    n = len(facs)
    if len(us) != n or n == 0:
        raise ValueError("one vector per factor, at least one factor")
    steps = [int(nsteps)] * n if isinstance(nsteps, int) else [int(k) for k in nsteps]
    if len(steps) != n:
        raise ValueError("one step count per problem")
    hs = (C.c_void_p * n)(*[f.h.value for f in facs])
    up = (C.c_void_p * n)(*[_dptr(u, f.N).value for f, u in zip(facs, us)])
    ks = (C.c_int64 * n)(*steps)
    st = Stats() if stats else None
    _check(lib.hlevy_step_batched(hs, up, ks, n, _refine(refine), C.byref(st) if st is not None else None,
                                  _stream(stream)), "hlevy_step_batched")
    return _stats_dict(st) if st is not None else None


def _refine(refine):
    if refine is None:
        return None
    r = Refine()
    r.tol = float(refine.get("tol", 0.0))
    r.sweeps = int(refine.get("sweeps", 2))
    r.check_every = int(refine.get("check_every", 0))
    r.max_sweeps = int(refine.get("max_sweeps", 0))
    return C.byref(r)


def fac_apply(fac: Fac, which: int, x, y, stream=None):
    """y = A x with the factor's per-step matrix: 0 = G (residual operator),
    1 = L^{-1}, 2 = U^{-1}."""
    _check(lib.hlevy_fac_apply(fac.h, int(which), _dptr(x, fac.N), _dptr(y, fac.N), _stream(stream)),
           "hlevy_fac_apply")


def solve(fac: Fac, b, x, refine=None, stats=False, stream=None):
    """Solve M x = b (hlevy_solve).  b, x: (N,) or (nrhs, N) contiguous
    float64 CUDA tensors; row c of a 2-D tensor is right-hand side c."""
    if b.shape != x.shape or b.dim() not in (1, 2) or b.shape[-1] != fac.N:
        raise ValueError("b and x must both be (N,) or (nrhs, N)")
    nrhs = 1 if b.dim() == 1 else int(b.shape[0])
    st = Stats() if stats else None
    _check(lib.hlevy_solve(fac.h, _dptr(b), _dptr(x), nrhs, fac.N, _refine(refine),
                           C.byref(st) if st is not None else None, _stream(stream)), "hlevy_solve")
    return _stats_dict(st) if st is not None else None


def solve_noalloc(fac: Fac, b, x, refine=None, stats=False, stream=None):
    """Solve M x = b for one right-hand side without device allocations
    (hlevy_solve_noalloc).  b, x: (N,) contiguous float64 CUDA tensors."""
    st = Stats() if stats else None
    _check(lib.hlevy_solve_noalloc(fac.h, _dptr(b, fac.N), _dptr(x, fac.N), _refine(refine),
                                   C.byref(st) if st is not None else None, _stream(stream)),
           "hlevy_solve_noalloc")
    return _stats_dict(st) if st is not None else None


def krylov_solve(fac: Fac, b, x, method: int = KRYLOV_CG, max_iter: int = 200, tol: float = 1e-12,
                 shift: float = 0.0, precondition: bool = True, use_guess: bool = False,
                 raise_not_converged: bool = True, op: Op | None = None, restart: int = 0, stream=None):
    """Solve (shift I - G) x = b by a Krylov iteration preconditioned with
    the factor (hlevy_krylov_solve).  b, x: (N,) contiguous float64 CUDA
    tensors.  Returns a dict with iterations, converged, rel_residual,
    seconds and the per-iteration relative residuals (history).  When tol
    is not met x holds the last iterate, and HlevyError (NOT_CONVERGED) is
    raised unless raise_not_converged is False.  op: the operator G of the
    iteration (default: the factor's own), e.g. a tighter compression of the
    same problem, which the factor then preconditions.  restart: GMRES
    cycle length (0: 30)."""
    o = KrylovOpts(int(method), int(max_iter), float(tol), float(shift), int(bool(precondition)),
                   int(bool(use_guess)), op.h.value if op is not None else None, int(restart), 0)
    st = KrylovStats()
    hist = (C.c_double * (int(max_iter) + 1))()
    rc = lib.hlevy_krylov_solve(fac.h, _dptr(b, fac.N), _dptr(x, fac.N), C.byref(o), C.byref(st), hist,
                                _stream(stream))
    if rc != -4 or raise_not_converged:   # -4: HLEVY_ERR_NOT_CONVERGED
        _check(rc, "hlevy_krylov_solve")
    return {"iterations": st.iterations, "converged": bool(st.converged), "rel_residual": st.rel_residual,
            "seconds": st.seconds, "history": [hist[i] for i in range(st.iterations + 1)]}


def step(fac: Fac, u, nsteps: int, g=None, phi=None, refine=None, stats=False, stream=None):
    gp = _dptr(g, fac.N) if g is not None else None
    php = None
    if g is not None:
        if phi is None or len(phi) != nsteps + 1:
            raise ValueError("phi must hold nsteps + 1 values")
        php = (C.c_double * (nsteps + 1))(*[float(v) for v in phi])
    st = Stats() if stats else None
    _check(lib.hlevy_step(fac.h, _dptr(u, fac.N), int(nsteps), gp, php, _refine(refine),
                          C.byref(st) if st is not None else None, _stream(stream)), "hlevy_step")
    if st is not None:
        return _stats_dict(st)
    return None


class Server:
    """Serving loop of the library (hlevy_server_*): submit requests, poll
    scheduling rounds, collect finished ids."""

    def __init__(self, prec: int = PREC_MIXED, lu_tol: float = 1e-6, sweeps: int = 1, chunk: int = 10,
                 max_active: int = 256, hbm_budget: int = 0, tol: float = 0.0, stream=None):
        cfg = ServerConfig(int(hbm_budget), int(prec), float(lu_tol), int(sweeps), int(chunk), int(max_active),
                           float(tol))
        h = C.c_void_p()
        _check(lib.hlevy_server_create(C.byref(cfg), _stream(stream), C.byref(h)), "hlevy_server_create")
        self.h = h
        self._keep = {}   # id -> (u0, u_out): the output must outlive the request

    def submit(self, prob: Problem, hp: HParams, dt: float, nsteps: int, u0, u_out) -> int:
        n = problem_N(prob)
        rid = C.c_int64()
        _check(lib.hlevy_server_submit(self.h, C.byref(prob), C.byref(hp), float(dt), int(nsteps),
                                       _dptr(u0, n), _dptr(u_out, n), C.byref(rid)), "hlevy_server_submit")
        self._keep[rid.value] = u_out
        return rid.value

    def poll(self, cap: int = 4096) -> list:
        ids = (C.c_int64 * cap)()
        nd = C.c_int32()
        _check(lib.hlevy_server_poll(self.h, ids, int(cap), C.byref(nd)), "hlevy_server_poll")
        out = [ids[i] for i in range(nd.value)]
        for i in out:
            self._keep.pop(i, None)
        return out

    def take_failed(self, cap: int = 4096) -> list:
        ids = (C.c_int64 * cap)()
        nd = C.c_int32()
        _check(lib.hlevy_server_take_failed(self.h, ids, int(cap), C.byref(nd)), "hlevy_server_take_failed")
        out = [ids[i] for i in range(nd.value)]
        for i in out:
            self._keep.pop(i, None)
        return out

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib.hlevy_server_stats_get(self.h, C.byref(st)), "hlevy_server_stats_get")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def __del__(self):
        if getattr(self, "h", None) and self.h.value and lib is not None:
            lib.hlevy_server_destroy(self.h)
            self.h = None
