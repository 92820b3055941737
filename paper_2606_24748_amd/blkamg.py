"""ctypes binding of libblkamg (argument marshalling only).

Every function here has the name of the C entry point it calls (include/blkamg.h)
and passes device pointers taken from torch tensors plus the current HIP stream.
No computation happens in Python: if the shared library is missing, importing this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BLKAMG_LIB") or os.path.join(_HERE, "libblkamg.so")

OK, ENOCONV, EINVAL, ENOMEM, EHIP, ESTATE, EBREAKDOWN, ENOTSPD = 0, 1, -1, -2, -3, -4, -5, -6
F64, F32, BF16 = 0, 1, 2
INSERT, ADD = 0, 1
FE_ATOMIC, FE_COLORED = 0, 1
AGG_GREEDY, AGG_LUBY = 0, 1
LUBY_SEED = 0x4D495332
EIG_LANCZOS, EIG_MLP = 0, 1
GUARD_SMOOTHER, GUARD_PCG = 0, 1
MLP_PARAMS, MLP_MODEL = 5122, 5150

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2606_24748_amd/build.py (or __graft_entry__.build())")

# torch is imported before the library is loaded: the library then binds to the HIP
# runtime torch has already loaded (same soname).  Loaded first, it would bring a second
# HIP/HSA runtime into the process, and torch would then report no GPU.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

_p = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_u64 = C.c_uint64
_f64 = C.c_double
_pi32 = C.POINTER(C.c_int32)


class Opts(C.Structure):
    _fields_ = [
        ("max_levels", C.c_int32),
        ("coarse_eq_limit", C.c_int32),
        ("strength_eps", C.c_double),
        ("cheb_degree", C.c_int32),
        ("cheb_lo", C.c_double),
        ("cheb_hi", C.c_double),
        ("lanczos_steps", C.c_int32),
        ("lanczos_seed", C.c_uint64),
        ("omega_scale", C.c_double),
        ("hier_dtype", C.c_int32),
        ("p_dtype", C.c_int32),
        ("pcg_graph_iters", C.c_int32),
        ("autotune_nrhs", C.c_int32),
        ("eig_mode", C.c_int32),
        ("agg_mode", C.c_int32),
        ("agg_seed", C.c_uint64),
        ("growth_steps", C.c_int32),
        ("eig_model", C.c_void_p),
        ("mlp_guard", C.c_int32),
        ("sym_spmv", C.c_int32),
        ("ap_residual", C.c_int32),
    ]


_SIG = {
    "blkamg_last_error": (C.c_char_p, []),
    "blkamg_version": (C.c_int, []),
    "blkamg_set_allocator": (C.c_int, [_p, _p, _p]),
    "bsr_create": (C.c_int, [_i32, _i32, _i32, _i32, _i64, _p, _p, _p, C.c_int, _p, C.POINTER(_p)]),
    "bsr_destroy": (C.c_int, [_p]),
    "bsr_mark_modified": (C.c_int, [_p]),
    "bsr_info": (C.c_int, [_p, _pi32, _pi32, _pi32, _pi32, C.POINTER(_i64), C.POINTER(C.c_int), C.POINTER(_u64)]),
    "bsr_arrays": (C.c_int, [_p, C.POINTER(_p), C.POINTER(_p), C.POINTER(_p)]),
    "bsr_spmv": (C.c_int, [_p, _f64, _p, _f64, _p, C.c_int, _i32, _p]),
    "bsr_spmv_t": (C.c_int, [_p, _f64, _p, _f64, _p, C.c_int, _i32, _p]),
    "bsr_spmv_sym": (C.c_int, [_p, _f64, _p, _f64, _p, C.c_int, _i32, _p]),
    "vcycle_apply_ex": (C.c_int, [_p, _p, _p, C.c_int, _i32, _p]),
    "bsr_autotune": (C.c_int, [_p, C.c_int, _i32, _p, _pi32]),
    "ptap_symbolic": (C.c_int, [_p, _p, C.POINTER(_p), _p]),
    "ptap_symbolic_ex": (C.c_int, [_p, _p, C.c_int, C.POINTER(_p), _p]),
    "ptap_numeric": (C.c_int, [_p, _p, _p, _p]),
    "ptap_plan_info": (C.c_int, [_p, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i32)]),
    "coo_plan_create": (C.c_int, [_i32, _i32, _i32, _i32, _i64, _p, _p, C.c_int, C.c_int, C.POINTER(_p),
                                  C.POINTER(_p), _p]),
    "coo_plan_destroy": (C.c_int, [_p]),
    "coo_plan_map": (C.c_int, [_p, C.POINTER(_p), C.POINTER(_p), C.POINTER(_i64), C.POINTER(_i64)]),
    "coo_assemble_blocked": (C.c_int, [_p, _p, C.c_int, C.c_int, _p, _p]),
    "sa_aggregate_device": (C.c_int, [_p, _p, C.c_uint64, _p, _pi32, _pi32, _p]),
    "sa_aggregate_device_noalloc": (C.c_int, [_p, _p, C.c_uint64, _p, _pi32, _pi32, _p]),
    "fe_q1_stream": (C.c_int, [_i64, _p, _p, _p, _p, _i64, _p, _p]),
    "fe_ebe_plan_create": (C.c_int, [_p, _i64, _p, _p, C.POINTER(_p)]),
    "fe_ebe_plan_info": (C.c_int, [_p, _pi32, C.POINTER(_i64)]),
    "fe_ebe_plan_destroy": (C.c_int, [_p]),
    "fe_q1_assemble_ebe": (C.c_int, [_p, _p, _p, _p, _p, _p, C.c_int, _p]),
    "blkamg_opts_default": (None, [C.POINTER(Opts)]),
    "sa_aggregate": (C.c_int, [_i32, _p, _p, _p, _p, _pi32]),
    "sa_tentative_device": (C.c_int, [_i32, _i32, _p, _i32, _p, _p, _p, _p]),
    "sa_setup_host": (C.c_int, [_i32, _p, _p, _p, _p, C.POINTER(Opts), C.POINTER(_p)]),
    "sa_result_info": (C.c_int, [_p, _pi32, C.POINTER(_i64), C.POINTER(_i64)]),
    "sa_result_arrays": (C.c_int, [_p] + [C.POINTER(_p)] * 7),
    "sa_result_free": (C.c_int, [_p]),
    "amg_setup": (C.c_int, [_p, _p, _p, C.POINTER(Opts), _p, C.POINTER(_p)]),
    "amg_setup_batched": (C.c_int, [_p, _i32, _p, _p, _p, C.POINTER(Opts), _p, C.POINTER(_p)]),
    "amg_destroy": (C.c_int, [_p]),
    "amg_num_levels": (C.c_int, [_p, _pi32]),
    "amg_num_instances": (C.c_int, [_p, _pi32]),
    "amg_instance_rows": (C.c_int, [_p, _i32, _p, _p, _p]),
    "amg_level": (C.c_int, [_p, _i32, C.POINTER(_p), C.POINTER(_p)]),
    "amg_aggregates": (C.c_int, [_p, _i32, _p]),
    "amg_lambdas": (C.c_int, [_p, _p]),
    "amg_galerkin_recompute": (C.c_int, [_p, _p]),
    "amg_smoother_refresh": (C.c_int, [_p, _p, _p]),
    "amg_hierarchy_create": (C.c_int, [_i32, _p, _p, C.POINTER(Opts), _p, C.POINTER(_p)]),
    "amg_hierarchy_update": (C.c_int, [_p, _p, _p]),
    "vcycle_apply": (C.c_int, [_p, _p, _p, _i32, _p]),
    "mlp_gemm_f32": (C.c_int, [_i32, _i32, _i32, _i32, _i32, _p, _i32, _p, _i32, _p, _i32, _p]),
    "mlp_forward": (C.c_int, [_p, _p, _i32, _p, _p, _p, _p]),
    "mlp_loss_grad": (C.c_int, [_p, _p, _p, _p, _p, _p, _i32, _p, _p, _p, _p]),
    "mlp_adam": (C.c_int, [_p, _p, _p, _p, _i32, _i32, C.c_float, C.c_float, C.c_float, C.c_float, _p]),
    "amg_features": (C.c_int, [_p, _p, _pi32, _p, _p, _p]),
    "amg_judge_lambdas": (C.c_int, [_p, _i32, _p, _p]),
    "amg_set_eig_model": (C.c_int, [_p, _p, _i32]),
    "amg_eig_status": (C.c_int, [_p, _p, _p, _p]),
    "amg_guard_status": (C.c_int, [_p, _pi32, _pi32]),
    "amg_setup_weights": (C.c_int, [_p, _p, _p, _p]),
    "pcg_solve": (C.c_int, [_p, _p, _p, _p, _f64, _i32, _i32, _pi32, C.POINTER(_f64), _p]),
}

for _name, (_res, _args) in _SIG.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class BlkAmgError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.blkamg_last_error().decode()
        super().__init__(f"{where} failed with status {code}: {msg}")
        self.code = code


def _check(code: int, where: str, allow=(OK,)) -> int:
    if code not in allow:
        raise BlkAmgError(code, where)
    return code


def exported_symbols():
    return list(_SIG)


def _stream(stream=None):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


_DT = {"float64": F64, "float32": F32, "bfloat16": BF16}


def dtype_code(t) -> int:
    return _DT[str(t.dtype).replace("torch.", "")]


def _dev_tensor(t, numel, dtypes, name):
    """Host-side check of a tensor handed to a kernel as a raw device pointer: a
    contiguous device tensor of one of `dtypes` with exactly `numel` elements.  A CPU
    tensor, a short vector or the wrong element type would otherwise make the kernel
    read or write out of bounds."""
    if t is None or not hasattr(t, "data_ptr"):
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype_code(t) not in dtypes:
        raise ValueError(f"{name} has dtype {t.dtype}, expected one of {[str(_torch_dtype(d)) for d in dtypes]}")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


def _vec_dtypes(mat_dtype):
    """Vector types a matrix of `mat_dtype` is applied to: F64 with F64 matrices, F32
    with F32 and BF16 matrices."""
    return (F64,) if mat_dtype == F64 else (F32,)


def _torch_dtype(code):
    import torch
    return {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}[code]


# ------------------------------------------------------------------------------
# handles
# ------------------------------------------------------------------------------
class Bsr:
    """Block sparse matrix handle.  Keeps the tensors it borrows alive."""

    def __init__(self, handle, keep=(), owned_by_lib=True, owner=None):
        self.h = C.c_void_p(handle) if not isinstance(handle, C.c_void_p) else handle
        self._keep = keep
        self._destroy = owned_by_lib and owner is None
        self._owner = owner
        self._shape = None

    def shape_info(self):
        """(nbr, nbc, bs_r, bs_c, dtype): fixed for the life of the handle, cached."""
        if self._shape is None:
            inf = self.info()
            self._shape = (inf["nbr"], inf["nbc"], inf["bs_r"], inf["bs_c"], inf["dtype"])
        return self._shape

    def __del__(self):
        if getattr(self, "_destroy", False) and self.h and _lib is not None:
            _lib.bsr_destroy(self.h)
            self.h = None

    def info(self):
        nbr, nbc, br, bc = _i32(), _i32(), _i32(), _i32()
        nnzb, dt, st = _i64(), C.c_int(), _u64()
        _check(_lib.bsr_info(self.h, nbr, nbc, br, bc, nnzb, dt, st), "bsr_info")
        return dict(nbr=nbr.value, nbc=nbc.value, bs_r=br.value, bs_c=bc.value, nnzb=nnzb.value,
                    dtype=dt.value, stamp=st.value)

    def arrays(self):
        """Copies of the device arrays as torch tensors (rowptr, colidx, values[nnzb, bs_r, bs_c])."""
        import torch
        inf = self.info()
        rp, ci, v = _p(), _p(), _p()
        _check(_lib.bsr_arrays(self.h, rp, ci, v), "bsr_arrays")
        nvals = inf["nnzb"] * inf["bs_r"] * inf["bs_c"]
        vals = _from_ptr(v.value, nvals, _torch_dtype(inf["dtype"]))
        return (_from_ptr(rp.value, inf["nbr"] + 1, torch.int32), _from_ptr(ci.value, inf["nnzb"], torch.int32),
                vals.view(inf["nnzb"], inf["bs_r"], inf["bs_c"]))


def _from_ptr(ptr, n, dtype):
    """Device-to-device copy of library-owned memory into a new torch tensor."""
    import torch
    out = torch.empty(n, dtype=dtype, device="cuda")
    if n == 0 or not ptr:
        return out
    torch.cuda.synchronize()
    rc = _hip().hipMemcpy(C.c_void_p(out.data_ptr()), C.c_void_p(ptr), C.c_size_t(n * out.element_size()), 3)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")
    return out


_HIP = None


def _hip():
    global _HIP
    if _HIP is None:
        _HIP = C.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.restype = C.c_int
        _HIP.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    return _HIP


def bsr_create(nbr, nbc, bs_r, bs_c, rowptr, colidx, val, stream=None) -> Bsr:
    """Wrap torch device tensors (int32 rowptr/colidx, float64/float32/bfloat16 values)."""
    h = _p()
    nnzb = int(colidx.numel())
    _check(_lib.bsr_create(nbr, nbc, bs_r, bs_c, nnzb, _ptr(rowptr), _ptr(colidx), _ptr(val),
                           dtype_code(val), _stream(stream), C.byref(h)), "bsr_create")
    return Bsr(h, keep=(rowptr, colidx, val))


def bsr_mark_modified(A: Bsr):
    _check(_lib.bsr_mark_modified(A.h), "bsr_mark_modified")


def _spmv_args(A: Bsr, x, y, nrhs, transpose):
    nbr, nbc, br, bc, dt = A.shape_info()
    if not 1 <= int(nrhs) <= 8:
        raise ValueError("nrhs must be in 1..8")
    nx, ny = (nbr * br, nbc * bc) if transpose else (nbc * bc, nbr * br)
    _dev_tensor(y, ny * nrhs, _vec_dtypes(dt), "y")
    _dev_tensor(x, nx * nrhs, (dtype_code(y),), "x")


def bsr_spmv(A: Bsr, alpha, x, beta, y, nrhs=1, stream=None):
    _spmv_args(A, x, y, nrhs, False)
    _check(_lib.bsr_spmv(A.h, float(alpha), _ptr(x), float(beta), _ptr(y), dtype_code(y), nrhs, _stream(stream)),
           "bsr_spmv")


def bsr_spmv_sym(A: Bsr, alpha, x, beta, y, nrhs=1, stream=None):
    """y = alpha S x + beta y, S the symmetric completion of A's upper triangle (A itself
    when A is symmetric), reading only the diagonal and upper blocks from memory."""
    _spmv_args(A, x, y, nrhs, False)
    _check(_lib.bsr_spmv_sym(A.h, float(alpha), _ptr(x), float(beta), _ptr(y), dtype_code(y), nrhs,
                             _stream(stream)), "bsr_spmv_sym")


def bsr_spmv_t(A: Bsr, alpha, x, beta, y, nrhs=1, stream=None):
    _spmv_args(A, x, y, nrhs, True)
    _check(_lib.bsr_spmv_t(A.h, float(alpha), _ptr(x), float(beta), _ptr(y), dtype_code(y), nrhs, _stream(stream)),
           "bsr_spmv_t")


def bsr_autotune(A: Bsr, vec_dtype=F64, nrhs=1, stream=None) -> int:
    """Time the compiled SpMV lane shapes of A and keep the fastest; returns G*8+U."""
    code = _i32()
    _check(_lib.bsr_autotune(A.h, int(vec_dtype), int(nrhs), _stream(stream), C.byref(code)), "bsr_autotune")
    return code.value


def ptap_symbolic(A: Bsr, P: Bsr, stream=None) -> Bsr:
    h = _p()
    _check(_lib.ptap_symbolic(A.h, P.h, C.byref(h), _stream(stream)), "ptap_symbolic")
    return Bsr(h, keep=(A, P))


PTAP_SYMMETRIC = 1
PTAP_HOST_SYMBOLIC = 2


def ptap_symbolic_ex(A: Bsr, P: Bsr, flags: int, stream=None) -> Bsr:
    h = _p()
    _check(_lib.ptap_symbolic_ex(A.h, P.h, int(flags), C.byref(h), _stream(stream)), "ptap_symbolic_ex")
    return Bsr(h, keep=(A, P))


def ptap_numeric(A: Bsr, P: Bsr, Cm: Bsr, stream=None):
    _check(_lib.ptap_numeric(A.h, P.h, Cm.h, _stream(stream)), "ptap_numeric")


def ptap_plan_info(Cm: Bsr) -> dict:
    """Sizes of the Galerkin plan attached to Cm: blocks of A P, the A P pass's and the
    R (A P) pass's block products (-1 without contribution lists), symmetric mode."""
    ap, pa, pc, sym = _i64(), _i64(), _i64(), _i32()
    _check(_lib.ptap_plan_info(Cm.h, C.byref(ap), C.byref(pa), C.byref(pc), C.byref(sym)), "ptap_plan_info")
    return {"ap_nnzb": ap.value, "ap_pairs": pa.value, "c_pairs": pc.value, "symmetric": bool(sym.value)}


class CooPlan:
    def __init__(self, h, n=None, block=None):
        self.h = h
        self.n = n            # coordinates the plan was made from (value stream length)
        self.block = block    # (bs_r, bs_c)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.coo_plan_destroy(self.h)
            self.h = None

    def index_map(self):
        import torch
        perm, seg, nv, nb = _p(), _p(), _i64(), _i64()
        _check(_lib.coo_plan_map(self.h, perm, seg, nv, nb), "coo_plan_map")
        return _from_ptr(perm.value, nv.value, torch.int32), _from_ptr(seg.value, nb.value + 1, torch.int32)


HOST, DEVICE = 0, 1


def coo_plan_create(nbr, nbc, bs_r, bs_c, i, j, val_dtype=F64, where=None, stream=None):
    """Coordinates as host int32 arrays (numpy; plan built on the host) or as int32 device
    tensors (plan built on the device); `where` defaults to the side the arrays live on.
    Returns (plan, A) with A library-owned."""
    on_dev = hasattr(i, "is_cuda") and i.is_cuda
    if where is None:
        where = DEVICE if on_dev else HOST
    if where == DEVICE:
        import torch
        for t, name in ((i, "i"), (j, "j")):
            if not (hasattr(t, "is_cuda") and t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous int32 device tensor for a device plan")
        if i.numel() != j.numel():
            raise ValueError("i and j differ in length")
        n = i.numel()
        pi, pj = _ptr(i), _ptr(j)
    else:
        i = np.ascontiguousarray(i, dtype=np.int32)
        j = np.ascontiguousarray(j, dtype=np.int32)
        if len(i) != len(j):
            raise ValueError("i and j differ in length")
        n = len(i)
        pi, pj = i.ctypes.data_as(_p), j.ctypes.data_as(_p)
    plan, A = _p(), _p()
    _check(_lib.coo_plan_create(nbr, nbc, bs_r, bs_c, n, pi, pj, int(where), val_dtype, C.byref(plan), C.byref(A),
                                _stream(stream) if where == DEVICE else None), "coo_plan_create")
    return CooPlan(plan, n, (bs_r, bs_c)), Bsr(A)


def coo_assemble_blocked(plan: CooPlan, vals, mode, A: Bsr, stream=None):
    _, _, br, bc, dt = A.shape_info()
    if plan.n is not None:
        _dev_tensor(vals, plan.n * br * bc, (dt,), "vals")
    if mode not in (INSERT, ADD):
        raise ValueError("mode must be INSERT or ADD")
    _check(_lib.coo_assemble_blocked(plan.h, _ptr(vals), dtype_code(vals), mode, A.h, _stream(stream)),
           "coo_assemble_blocked")


def sa_aggregate_device(A: Bsr, dirichlet=None, seed=LUBY_SEED, stream=None):
    """Distance-2 aggregation of A's block graph on the device (Luby rounds).
    Returns (agg device int32 tensor, n_agg, rounds); dirichlet: host bool/uint8 or None."""
    import torch
    n = A.info()["nbr"]
    agg = torch.empty(n, dtype=torch.int32, device="cuda")
    d = None
    if dirichlet is not None:
        d = torch.as_tensor(np.ascontiguousarray(dirichlet, dtype=np.uint8)).cuda()
        if d.numel() != n:
            raise ValueError("dirichlet must have one flag per block row")
    na, nr = _i32(), _i32()
    _check(_lib.sa_aggregate_device(A.h, _ptr(d), seed, _ptr(agg), C.byref(na), C.byref(nr), _stream(stream)),
           "sa_aggregate_device")
    return agg, na.value, nr.value


def sa_aggregate_device_noalloc(A: Bsr, d_dirichlet, d_agg, seed=LUBY_SEED, stream=None):
    """sa_aggregate_device on the library's static scratch, writing into caller tensors:
    d_dirichlet (device uint8 [nbr] or None) and d_agg (device int32 [nbr]).  Allocates
    nothing on the device.  Returns (n_agg, rounds)."""
    n = A.info()["nbr"]
    if not (hasattr(d_agg, "is_cuda") and d_agg.is_cuda and d_agg.is_contiguous() and d_agg.numel() == n
            and str(d_agg.dtype) == "torch.int32"):
        raise ValueError("d_agg must be a contiguous device int32 tensor with one entry per block row")
    if d_dirichlet is not None and not (d_dirichlet.is_cuda and d_dirichlet.is_contiguous()
                                        and d_dirichlet.numel() == n and str(d_dirichlet.dtype) == "torch.uint8"):
        raise ValueError("d_dirichlet must be a contiguous device uint8 tensor with one flag per block row")
    na, nr = _i32(), _i32()
    _check(_lib.sa_aggregate_device_noalloc(A.h, _ptr(d_dirichlet), seed, _ptr(d_agg), C.byref(na), C.byref(nr),
                                            _stream(stream)), "sa_aggregate_device_noalloc")
    return na.value, nr.value


def sa_tentative_device(agg, n_agg, B_null, stream=None):
    """P~ values [nbr, bs, 6] and the coarse near-null space [n_agg, 6, 6] from device
    tensors agg (int32 [nbr]) and B_null (float64 [nbr, bs, 6])."""
    import torch
    nbr = agg.numel()
    if B_null.dim() != 3 or B_null.shape[0] != nbr or B_null.shape[2] != 6:
        raise ValueError("B_null must be [nbr, bs, 6]")
    bs = B_null.shape[1]
    if agg.dtype != torch.int32 or not agg.is_cuda or not agg.is_contiguous():
        raise ValueError("agg must be a contiguous int32 device tensor")
    _dev_tensor(B_null, nbr * bs * 6, (F64,), "B_null")
    pt = torch.empty(nbr, bs, 6, dtype=torch.float64, device="cuda")
    bc = torch.empty(max(n_agg, 0), 6, 6, dtype=torch.float64, device="cuda")
    _check(_lib.sa_tentative_device(nbr, bs, _ptr(agg), int(n_agg), _ptr(B_null), _ptr(pt), _ptr(bc),
                                    _stream(stream)), "sa_tentative_device")
    return pt, bc


def _fe_inputs(elem_nodes, coords, lam, mu, check_nodes=True):
    """Check the element inputs: contiguous device tensors, int32 [n_elem, 8] nodes,
    float64 [n_nodes, 3] coordinates, float64 [n_elem] Lame parameters; with
    check_nodes, also that every node indexes a row of coords (one reduction and a
    sync: callers that time the kernels check once and then pass False)."""
    import torch
    want = ((elem_nodes, torch.int32), (coords, torch.float64), (lam, torch.float64), (mu, torch.float64))
    for t, dt in want:
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"expected a contiguous device tensor of {dt}")
    n_elem = elem_nodes.shape[0]
    if elem_nodes.shape != (n_elem, 8) or coords.dim() != 2 or coords.shape[1] != 3 or \
            lam.numel() != n_elem or mu.numel() != n_elem:
        raise ValueError("element input shapes do not match")
    if check_nodes and n_elem > 0:
        lo, hi = int(elem_nodes.min()), int(elem_nodes.max())
        if lo < 0 or hi >= coords.shape[0]:
            raise ValueError("an element node does not index a row of coords")
    return n_elem


def fe_q1_stream(elem_nodes, coords, lam, mu, out, n_identity=0, stream=None, check_nodes=True):
    """Element stiffness blocks of trilinear hexahedra into the blocked COO value stream
    `out` (device F64, [n_elem * 64 + n_identity, 3, 3]); all inputs device tensors."""
    import torch
    n_elem = _fe_inputs(elem_nodes, coords, lam, mu, check_nodes)
    if out.dtype != torch.float64 or not out.is_contiguous() or out.numel() != (n_elem * 64 + n_identity) * 9:
        raise ValueError("out must be a contiguous float64 tensor of (n_elem * 64 + n_identity) * 9 values")
    _check(_lib.fe_q1_stream(n_elem, _ptr(elem_nodes), _ptr(coords), _ptr(lam), _ptr(mu), n_identity, _ptr(out),
                             _stream(stream)), "fe_q1_stream")


class FePlan:
    def __init__(self, h, A):
        self.h = h
        self._A = A

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fe_ebe_plan_destroy(self.h)
            self.h = None

    def info(self):
        nc, nb = _i32(), _i64()
        _check(_lib.fe_ebe_plan_info(self.h, C.byref(nc), C.byref(nb)), "fe_ebe_plan_info")
        return {"n_colors": nc.value, "bytes": nb.value}


def fe_ebe_plan_create(A: Bsr, elem_nodes: np.ndarray, dirichlet=None) -> FePlan:
    en = np.ascontiguousarray(elem_nodes, dtype=np.int32)
    dd = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
    h = _p()
    _check(_lib.fe_ebe_plan_create(A.h, en.shape[0], en.ctypes.data_as(_p),
                                   dd.ctypes.data_as(_p) if dd is not None else None, C.byref(h)),
           "fe_ebe_plan_create")
    return FePlan(h, A)


def fe_q1_assemble_ebe(P: FePlan, A: Bsr, elem_nodes, coords, lam, mu, mode=FE_COLORED, stream=None,
                       check_nodes=True):
    _fe_inputs(elem_nodes, coords, lam, mu, check_nodes)
    _check(_lib.fe_q1_assemble_ebe(P.h, A.h, _ptr(elem_nodes), _ptr(coords), _ptr(lam), _ptr(mu), mode,
                                   _stream(stream)), "fe_q1_assemble_ebe")


def blkamg_opts_default() -> Opts:
    o = Opts()
    _lib.blkamg_opts_default(C.byref(o))
    return o


def sa_aggregate(rowptr: np.ndarray, colidx: np.ndarray, dirichlet=None):
    """Host-only greedy aggregation; returns (agg int32[nbr], n_agg)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    nbr = len(rowptr) - 1
    agg = np.empty(nbr, dtype=np.int32)
    n = _i32()
    d = None
    if dirichlet is not None:
        dd = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        d = dd.ctypes.data_as(_p)
    _check(_lib.sa_aggregate(nbr, rowptr.ctypes.data_as(_p), colidx.ctypes.data_as(_p), d,
                             agg.ctypes.data_as(_p), C.byref(n)), "sa_aggregate")
    return agg, n.value


def sa_setup_host(rowptr: np.ndarray, colidx: np.ndarray, coords: np.ndarray, dirichlet=None) -> dict:
    """Host setup of one aggregation level from the fine block pattern (sa_setup_host):
    copies of agg, the tentative prolongator (pt_rowptr, pt_colidx, pt_val [nnzb,3,6]),
    the coarse near-null space bc [n_agg,6,6] and the smoothed-prolongator pattern."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    n = len(rowptr) - 1
    d = None
    if dirichlet is not None:
        dd = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        d = dd.ctypes.data_as(_p)
    h = _p()
    _check(_lib.sa_setup_host(n, rowptr.ctypes.data_as(_p), colidx.ctypes.data_as(_p), d,
                              coords.ctypes.data_as(_p), None, C.byref(h)), "sa_setup_host")
    try:
        na, pn, sn = _i32(), _i64(), _i64()
        _check(_lib.sa_result_info(h, C.byref(na), C.byref(pn), C.byref(sn)), "sa_result_info")
        ptrs = [_p() for _ in range(7)]
        _check(_lib.sa_result_arrays(h, *[C.byref(q) for q in ptrs]), "sa_result_arrays")

        def arr(q, count, ctype, dtype):
            if count == 0:
                return np.zeros(0, dtype=dtype)
            return np.ctypeslib.as_array(C.cast(q, C.POINTER(ctype)), shape=(count,)).astype(dtype, copy=True)

        out = {"n_agg": na.value,
               "agg": arr(ptrs[0], n, C.c_int32, np.int32),
               "pt_rowptr": arr(ptrs[1], n + 1, C.c_int32, np.int32),
               "pt_colidx": arr(ptrs[2], pn.value, C.c_int32, np.int32),
               "pt_val": arr(ptrs[3], pn.value * 18, C.c_double, np.float64).reshape(pn.value, 3, 6),
               "bc": arr(ptrs[4], na.value * 36, C.c_double, np.float64).reshape(na.value, 6, 6),
               "sp_rowptr": arr(ptrs[5], n + 1, C.c_int32, np.int32),
               "sp_colidx": arr(ptrs[6], sn.value, C.c_int32, np.int32)}
    finally:
        _lib.sa_result_free(h)
    return out


class Amg:
    def __init__(self, h, keep=()):
        self.h = h
        self._keep = keep

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.amg_destroy(self.h)
            self.h = None

    def num_levels(self) -> int:
        n = _i32()
        _check(_lib.amg_num_levels(self.h, C.byref(n)), "amg_num_levels")
        return n.value

    def level(self, l):
        A, P = _p(), _p()
        _check(_lib.amg_level(self.h, l, C.byref(A), C.byref(P)), "amg_level")
        return (Bsr(A, owner=self), Bsr(P, owner=self) if P.value else None)

    def num_instances(self) -> int:
        n = _i32()
        _check(_lib.amg_num_instances(self.h, C.byref(n)), "amg_num_instances")
        return n.value

    def instance_rows(self, l):
        """(row0, nrows, state) per instance on level l; state 0 absent, 1 smoothed, 2 coarsest."""
        k = self.num_instances()
        r0, nr, st = (np.zeros(k, dtype=np.int32) for _ in range(3))
        _check(_lib.amg_instance_rows(self.h, l, r0.ctypes.data_as(_p), nr.ctypes.data_as(_p),
                                      st.ctypes.data_as(_p)), "amg_instance_rows")
        return r0, nr, st

    def aggregates(self, l):
        _, nr, st = self.instance_rows(l)
        agg = np.empty(int(nr[st == 1].sum()), dtype=np.int32)
        _check(_lib.amg_aggregates(self.h, l, agg.ctypes.data_as(_p)), "amg_aggregates")
        return agg

    def lambdas(self):
        """lambda_hat [n_levels - 1] for one instance, [n_levels - 1][n_inst] for a batch."""
        k = self.num_instances()
        lam = np.zeros((max(self.num_levels() - 1, 0), k))
        if lam.size:
            _check(_lib.amg_lambdas(self.h, lam.ctypes.data_as(_p)), "amg_lambdas")
        return lam[:, 0] if k == 1 else lam


def amg_setup(A0: Bsr, coords: np.ndarray, dirichlet=None, opts: Opts | None = None, stream=None) -> Amg:
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    d = None
    dd = None
    if dirichlet is not None:
        dd = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        d = dd.ctypes.data_as(_p)
    o = opts or blkamg_opts_default()
    h = _p()
    _check(_lib.amg_setup(A0.h, coords.ctypes.data_as(_p), d, C.byref(o), _stream(stream), C.byref(h)),
           "amg_setup")
    return Amg(h, keep=(A0,))


def amg_setup_batched(A0: Bsr, inst_row0, coords: np.ndarray, dirichlet=None, opts: Opts | None = None,
                      stream=None) -> Amg:
    """Hierarchy of a block-diagonal batch: instance t owns block rows [inst_row0[t], inst_row0[t+1])."""
    row0 = np.ascontiguousarray(inst_row0, dtype=np.int32)
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    d = None
    dd = None
    if dirichlet is not None:
        dd = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        d = dd.ctypes.data_as(_p)
    o = opts or blkamg_opts_default()
    h = _p()
    _check(_lib.amg_setup_batched(A0.h, len(row0) - 1, row0.ctypes.data_as(_p), coords.ctypes.data_as(_p), d,
                                  C.byref(o), _stream(stream), C.byref(h)), "amg_setup_batched")
    return Amg(h, keep=(A0,))


def amg_galerkin_recompute(M: Amg, stream=None):
    _check(_lib.amg_galerkin_recompute(M.h, _stream(stream)), "amg_galerkin_recompute")


def _lambda_arg(M: Amg, lambdas, dtype):
    """Host array [n_levels - 1][n_inst] of `dtype` (kept alive by the caller) and its pointer."""
    if lambdas is None:
        return None, None
    arr = np.ascontiguousarray(lambdas, dtype=dtype)
    want = max(M.num_levels() - 1, 0) * M.num_instances()
    if arr.size != want:
        raise ValueError(f"lambdas has {arr.size} entries, the hierarchy needs {want}")
    return arr, arr.ctypes.data_as(_p)


def amg_smoother_refresh(M: Amg, lambdas=None, stream=None):
    arr, lam = _lambda_arg(M, lambdas, np.float64)
    _check(_lib.amg_smoother_refresh(M.h, lam, _stream(stream)), "amg_smoother_refresh")
    del arr


def amg_hierarchy_create(A: list, P: list, opts: Opts | None = None, stream=None) -> Amg:
    """Hierarchy from caller operators A[0..L-1] (F64; 3x3 then 6x6 blocks) and prolongators
    P[0..L-2] (F64, copied).  The A handles are kept alive by the returned object."""
    n = len(A)
    if len(P) != max(n - 1, 0):
        raise ValueError("need len(P) == len(A) - 1")
    a_arr = (_p * n)(*[x.h for x in A])
    p_arr = (_p * max(n - 1, 1))(*([x.h for x in P] or [None]))
    o = opts or blkamg_opts_default()
    h = _p()
    _check(_lib.amg_hierarchy_create(n, a_arr, p_arr if P else None, C.byref(o), _stream(stream), C.byref(h)),
           "amg_hierarchy_create")
    return Amg(h, keep=tuple(A))


def amg_hierarchy_update(M: Amg, lambdas=None, stream=None):
    """Smoother refresh with lambda_hat given in single precision ([n_levels - 1][n_inst]) or estimated."""
    arr, lam = _lambda_arg(M, lambdas, np.float32)
    _check(_lib.amg_hierarchy_update(M.h, lam, _stream(stream)), "amg_hierarchy_update")
    del arr


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)
_allocator_keep = []  # every callback pair ever installed: buffers return to the pair that made them


def blkamg_set_allocator(alloc_fn=None, free_fn=None, ctx=None):
    """Route the library's device allocations through alloc_fn(bytes, ctx) -> int pointer and
    free_fn(ptr, bytes, ctx) (Python callables), or back to hipMalloc/hipFree when both are None."""
    if alloc_fn is None and free_fn is None:
        _check(_lib.blkamg_set_allocator(None, None, None), "blkamg_set_allocator")
        return
    a = _ALLOC_FN(alloc_fn) if alloc_fn is not None else None
    f = _FREE_FN(free_fn) if free_fn is not None else None
    _check(_lib.blkamg_set_allocator(C.cast(a, _p) if a else None, C.cast(f, _p) if f else None, ctx),
           "blkamg_set_allocator")
    _allocator_keep.append((a, f))


def use_torch_allocator(enable=True):
    """Take the library's device memory from PyTorch's caching allocator (current device and stream)."""
    if not enable:
        blkamg_set_allocator()
        return

    def alloc(nbytes, _ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:
            return None

    def free(ptr, _nbytes, _ctx):
        torch.cuda.caching_allocator_delete(ptr)

    blkamg_set_allocator(alloc, free)


def _fine_dofs(M: Amg) -> int:
    n = getattr(M, "_fine_dofs", None)
    if n is None:
        A0, _ = M.level(0)
        nbr, _, br, _, _ = A0.shape_info()
        n = M._fine_dofs = nbr * br
    return n


def vcycle_apply(M: Amg, r, z, nrhs=1, stream=None):
    """z = M^-1 r.  FP64 vectors on any hierarchy; FP32 vectors (through vcycle_apply_ex)
    on an F32 hierarchy."""
    n = _fine_dofs(M) * int(nrhs)
    _dev_tensor(r, n, (F64, F32), "r")
    _dev_tensor(z, n, (dtype_code(r),), "z")
    if dtype_code(r) == F64:
        _check(_lib.vcycle_apply(M.h, _ptr(r), _ptr(z), nrhs, _stream(stream)), "vcycle_apply")
    else:
        _check(_lib.vcycle_apply_ex(M.h, _ptr(r), _ptr(z), F32, nrhs, _stream(stream)), "vcycle_apply_ex")


def pcg_solve(A: Bsr, M: Amg, b, x, rtol=1e-8, maxit=1000, nrhs=1, stream=None):
    """Returns (status, iterations, relative residual); status OK or ENOCONV.  For one
    instance and nrhs = 1 the last two are scalars, otherwise int32 / float64 arrays
    [n_inst][nrhs]."""
    nbr, _, br, _, _ = A.shape_info()
    _dev_tensor(b, nbr * br * int(nrhs), (F64,), "b")
    _dev_tensor(x, nbr * br * int(nrhs), (F64,), "x")
    k = M.num_instances()
    it = np.zeros(k * nrhs, dtype=np.int32)
    rr = np.zeros(k * nrhs, dtype=np.float64)
    code = _lib.pcg_solve(A.h, M.h, _ptr(b), _ptr(x), float(rtol), int(maxit), int(nrhs), it.ctypes.data_as(_pi32),
                          rr.ctypes.data_as(C.POINTER(_f64)), _stream(stream))
    _check(code, "pcg_solve", allow=(OK, ENOCONV))
    if k == 1 and nrhs == 1:
        return code, int(it[0]), float(rr[0])
    return code, it.reshape(k, nrhs), rr.reshape(k, nrhs)


# ------------------------------------------------------------------------------
# learned eigenbound
# ------------------------------------------------------------------------------
def mlp_gemm_f32(a, b, c, trans_a=False, trans_b=False, stream=None):
    """c = op(a) op(b) for 2-D float32 device tensors (row-major, contiguous)."""
    m = a.shape[1] if trans_a else a.shape[0]
    k = a.shape[0] if trans_a else a.shape[1]
    n = b.shape[0] if trans_b else b.shape[1]
    _check(_lib.mlp_gemm_f32(int(trans_a), int(trans_b), m, n, k, _ptr(a), a.shape[1], _ptr(b), b.shape[1], _ptr(c),
                             c.shape[1], _stream(stream)), "mlp_gemm_f32")


def mlp_forward(theta, x, h1, h2, y, stream=None):
    _check(_lib.mlp_forward(_ptr(theta), _ptr(x), x.shape[0], _ptr(h1), _ptr(h2), _ptr(y), _stream(stream)),
           "mlp_forward")


def mlp_loss_grad(theta, x, h1, h2, y, t, work, grad, loss=None, stream=None):
    _check(_lib.mlp_loss_grad(_ptr(theta), _ptr(x), _ptr(h1), _ptr(h2), _ptr(y), _ptr(t), x.shape[0], _ptr(work),
                              _ptr(grad), _ptr(loss), _stream(stream)), "mlp_loss_grad")


def mlp_adam(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(_lib.mlp_adam(_ptr(theta), _ptr(grad), _ptr(m), _ptr(v), theta.numel(), int(step), float(lr), float(beta1),
                         float(beta2), float(eps), _stream(stream)), "mlp_adam")


def amg_features(M: Amg, stream=None):
    """(features [n_samples][12] float32 device tensor, level[n], instance[n])."""
    import torch
    n = _i32()
    _check(_lib.amg_features(M.h, None, C.byref(n), None, None, _stream(stream)), "amg_features")
    lev = np.zeros(n.value, dtype=np.int32)
    inst = np.zeros(n.value, dtype=np.int32)
    feat = torch.zeros(max(n.value, 1), 12, dtype=torch.float32, device="cuda")
    _check(_lib.amg_features(M.h, _ptr(feat), C.byref(n), lev.ctypes.data_as(_p), inst.ctypes.data_as(_p),
                             _stream(stream)), "amg_features")
    return feat[:n.value], lev, inst


def amg_judge_lambdas(M: Amg, k=50, stream=None):
    """[n_levels - 1][n_inst] reference lambda_max (k-step reorthogonalised Lanczos)."""
    lam = np.zeros((max(M.num_levels() - 1, 0), M.num_instances()))
    if lam.size:
        _check(_lib.amg_judge_lambdas(M.h, int(k), lam.ctypes.data_as(_p), _stream(stream)), "amg_judge_lambdas")
    return lam


def amg_set_eig_model(M: Amg, model: np.ndarray):
    model = np.ascontiguousarray(model, dtype=np.float32)
    _check(_lib.amg_set_eig_model(M.h, model.ctypes.data_as(_p), model.size), "amg_set_eig_model")


def amg_eig_status(M: Amg):
    """(fallback[n_levels-1], growth[n_levels-1][n_inst], omega[n_levels-1][n_inst])."""
    nl = max(M.num_levels() - 1, 0)
    k = M.num_instances()
    fb = np.zeros(nl, dtype=np.int32)
    g = np.zeros((nl, k))
    om = np.zeros((nl, k))
    _check(_lib.amg_eig_status(M.h, fb.ctypes.data_as(_p), g.ctypes.data_as(_p), om.ctypes.data_as(_p)),
           "amg_eig_status")
    return fb, g, om


def amg_guard_status(M: Amg):
    """(armed, restarts) of the deferred guard (mlp_guard = GUARD_PCG)."""
    a, r = _i32(), _i32()
    _check(_lib.amg_guard_status(M.h, C.byref(a), C.byref(r)), "amg_guard_status")
    return bool(a.value), r.value


def amg_setup_weights(M: Amg):
    """What the cold setup used per smoothed level: (lambda[n_levels-1][n_inst],
    omega[n_levels-1][n_inst], learned[n_levels-1]) with learned = 1 where the network
    supplied them."""
    nl = max(M.num_levels() - 1, 0)
    k = M.num_instances()
    lam = np.zeros((nl, k))
    om = np.zeros((nl, k))
    le = np.zeros(nl, dtype=np.int32)
    _check(_lib.amg_setup_weights(M.h, lam.ctypes.data_as(_p), om.ctypes.data_as(_p), le.ctypes.data_as(_p)),
           "amg_setup_weights")
    return lam, om, le


def opts_with_model(opts: Opts, model: np.ndarray):
    """Point opts.eig_model at a host float32 copy of `model` (BLKAMG_MLP_MODEL floats).
    Returns the array, which must stay alive until the setup call has returned (the
    library copies it)."""
    arr = np.ascontiguousarray(model, dtype=np.float32)
    if arr.size != MLP_MODEL:
        raise ValueError(f"a model has {MLP_MODEL} floats, got {arr.size}")
    opts.eig_model = arr.ctypes.data
    return arr
