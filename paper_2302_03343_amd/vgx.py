"""ctypes binding of libvgx.so (the C ABI in include/vgx.h).

Argument marshalling only: every function below has the name of the C entry
point it calls, converts torch tensors to device pointers and numpy arrays to
host pointers, passes the current HIP stream, and raises VgxError on a
non-zero status.  No arithmetic of the method happens here.  Importing this
module fails loudly if the compiled library is missing; there is no fallback.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libvgx.so")

VGX_OK, VGX_EINVAL, VGX_ENOMEM, VGX_EDEVICE, VGX_ERANGE, VGX_ENUMERIC, VGX_EFALLBACK, VGX_ESTATE = range(8)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ERANGE", 5: "ENUMERIC",
                6: "EFALLBACK", 7: "ESTATE"}
GAUSS, GENZ_OSC, GENZ_PEAK, TTBAR, DRELLYAN, SINGLETOP = 0, 1, 2, 3, 4, 5
F64, F32 = 0, 1
EXTRAP_ERROR, EXTRAP_FREEZE, EXTRAP_CONTINUE = 0, 1, 2
OPERANDS_BF16, OPERANDS_F32 = 0, 1
MAX_DIM, MAX_BINS = 12, 256


class VgxError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libvgx.so not found at {LIB_PATH}; build it with `python -m paper_2302_03343_amd.build` "
        "(the HIP path has no CPU fallback)")

# One HIP runtime per process: PyTorch ships its own copy of the HIP runtime
# (same soname as the system one).  Loading PyTorch first makes the library's
# dependency resolve to that already-loaded copy, so device memory, streams
# and synchronisation are shared with the caller's tensors; loaded the other
# way round, the process would hold two runtimes that do not see each other's
# streams (and the library's launches would not run on the caller's queues).
try:
    import torch  # noqa: F401  (for its HIP runtime)
except ImportError:  # C-ABI use without PyTorch: the system runtime
    torch = None

_lib = C.CDLL(LIB_PATH)
_vp = C.c_void_p
_i32, _i64, _u32, _u64, _f32, _f64 = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_float, C.c_double


class IterResult(C.Structure):
    _fields_ = [("mean", _f64), ("var", _f64), ("s1", _f64), ("s2", _f64), ("n", _i64)]

    def as_dict(self):
        return dict(mean=self.mean, var=self.var, s1=self.s1, s2=self.s2, n=self.n)


class VegasCfg(C.Structure):
    _fields_ = [("kind", _i32), ("dim", _i32), ("n_bins", _i32), ("alpha", _f64), ("seed", _u64),
                ("stream_id", _u32), ("prec", _i32), ("params", C.POINTER(_f64)), ("n_params", _i32),
                ("pdf", _vp)]


class PdfDesc(C.Structure):
    _fields_ = [("n_x", _i32), ("n_sub", _i32), ("n_flav", _i32), ("x_knots", C.POINTER(_f64)),
                ("nq_per_sub", C.POINTER(_i32)), ("q2_knots", C.POINTER(_f64)), ("xf", C.POINTER(_f64))]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_S = C.c_int  # vgx_status


class LheInit(C.Structure):
    _fields_ = [("beam_id", _i32 * 2), ("beam_energy", _f64 * 2), ("pdf_group", _i32 * 2), ("pdf_set", _i32 * 2),
                ("weight_mode", _i32), ("xsec", _f64), ("xsec_err", _f64), ("xmax", _f64), ("proc_id", _i32)]


class LheEventInfo(C.Structure):
    _fields_ = [("sqrt_s", _f64), ("weight", _f64), ("scale", _f64), ("aqed", _f64), ("aqcd", _f64),
                ("proc_id", _i32)]
_c = {}
for _name, _res, _args in [
    ("vgx_last_error", C.c_char_p, []),
    ("vgx_version", C.c_char_p, []),
    ("pdf_create", _S, [C.POINTER(PdfDesc), _vp, C.POINTER(_vp)]),
    ("pdf_interp", _S, [_vp, _i64, _vp, _vp, _i32, _vp, _vp]),
    ("pdf_create_set", _S, [C.POINTER(PdfDesc), _i32, _vp, C.POINTER(_vp)]),
    ("pdf_interp_members", _S, [_vp, _i64, _vp, _vp, _i32, _vp, _vp]),
    ("pdf_shape", _S, [_vp, C.POINTER(_i32), C.POINTER(_i32)]),
    ("pdf_out_of_range", _S, [_vp, _vp, C.POINTER(_i64)]),
    ("pdf_bounds", _S, [_vp, C.POINTER(_f64), C.POINTER(_f64), C.POINTER(_f64), C.POINTER(_f64)]),
    ("pdf_set_extrapolation", _S, [_vp, _i32]),
    ("pdf_set_alphas", _S, [_vp, _i32, C.POINTER(_f64), C.POINTER(_f64), _vp]),
    ("pdf_alphas", _S, [_vp, _i64, _vp, _vp, _vp]),
    ("pdf_destroy", None, [_vp]),
    ("rambo_generate", _S, [_i32, C.POINTER(_f64), _f64, _u64, _u32, _u32, _i64, _i64, _vp, _vp, _vp]),
    ("unweight", _S, [_i64, _vp, _f64, _u64, _u32, _u32, _vp, C.POINTER(_i64), C.POINTER(_f64), _vp]),
    ("unweight_noalloc", _S, [_i64, _vp, _f64, _u64, _u32, _u32, _vp, C.POINTER(_i64), C.POINTER(_f64), _vp]),
    ("lhe_open", _S, [C.c_char_p, C.POINTER(LheInit), C.POINTER(_vp)]),
    ("lhe_write_events", _S, [_vp, _i32, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_f64), C.POINTER(LheEventInfo),
                              _i64, _vp, _vp, _i64, _vp]),
    ("lhe_write_events_host", _S, [_vp, _i32, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_f64),
                                   C.POINTER(LheEventInfo), _i64, C.POINTER(_f64)]),
    ("lhe_flush", _S, [_vp, C.POINTER(_i64)]),
    ("lhe_close", _S, [_vp]),
    ("vegas_create", _S, [C.POINTER(VegasCfg), _vp, C.POINTER(_vp)]),
    ("vegas_iterate", _S, [_vp, _i64, _i32, C.POINTER(IterResult)]),
    ("vegas_iterate_async", _S, [_vp, _i64, _i32]),
    ("vegas_refine", _S, [_vp]),
    ("vegas_result", _S, [_vp, C.POINTER(_f64), C.POINTER(_f64), C.POINTER(_f64), C.POINTER(_i32)]),
    ("vegas_results", _S, [_vp, C.POINTER(IterResult), _i32, C.POINTER(_i32)]),
    ("vegas_reset_results", _S, [_vp]),
    ("vegas_get_grid", _S, [_vp, C.POINTER(_f64)]),
    ("vegas_set_grid", _S, [_vp, C.POINTER(_f64)]),
    ("vegas_get_hist", _S, [_vp, C.POINTER(_f64)]),
    ("vegas_sample", _S, [_vp, _i64, _i64, _i32, _vp, _vp]),
    ("vegas_iterate_points", _S, [_vp, _i64, _vp, _vp, C.POINTER(IterResult)]),
    ("vegas_stream", _vp, [_vp]),
    ("vegas_shape", _S, [_vp, C.POINTER(_i32), C.POINTER(_i32)]),
    ("vegas_set_timing", _S, [_vp, _i32]),
    ("vegas_kernel_time", _S, [_vp, C.POINTER(_f64), C.POINTER(_i64)]),
    ("vegas_destroy", None, [_vp]),
]:
    _c[_name] = _sig(_name, _res, *_args)


def _optional(name, res, *args):
    if hasattr(_lib, name):
        _c[name] = _sig(name, res, *args)


_optional("batch_create", _S, C.POINTER(_vp), _i32, C.POINTER(_i64), _i32, _i32, _vp, C.POINTER(_vp))
_optional("batch_iterate", _S, _vp, _i32, C.POINTER(IterResult))
_optional("batch_config", _S, _vp, C.POINTER(_i32), C.POINTER(_i32))
_optional("batch_destroy", None, _vp)
_optional("flow_num_params", _i64, _i32, _i32, _i32, _i32)
_optional("flow_shape", _S, _vp, C.POINTER(_i32), C.POINTER(_i64))
_optional("flow_param_layout", _S, _i32, _i32, _i32, _i32, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i64), _i32,
          C.POINTER(_i32))
_optional("flow_create", _S, _i32, _i32, _i32, _i32, C.POINTER(_f32), _i64, _vp, C.POINTER(_vp))
_optional("flow_sample", _S, _vp, _i64, _u64, _u32, _i32, _vp, _vp, _vp)
_optional("flow_density", _S, _vp, _i64, _vp, _vp, _vp, _vp)
_optional("flow_loss_grad", _S, _vp, _i64, _vp, _vp, C.POINTER(_f64), C.POINTER(_f32))
_optional("flow_train_step", _S, _vp, _i64, _vp, _vp, _f32, C.POINTER(_f64))
_optional("flow_adam", _S, _vp, _vp, _f32)
_optional("flow_get_params", _S, _vp, C.POINTER(_f32), _i64, C.POINTER(_i64))
_optional("flow_set_params", _S, _vp, C.POINTER(_f32), _i64)
_optional("flow_set_operands", _S, _vp, _i32)
_optional("flow_vegas_iterate", _S, _vp, _vp, _i64, _u64, _u32, _i32, C.POINTER(IterResult))
_optional("flow_destroy", None, _vp)

EXPORTED = sorted(_c)


def _check(st, where):
    if st != VGX_OK:
        msg = _c["vgx_last_error"]().decode(errors="replace")
        raise VgxError(st, where, msg)


def last_error():
    return _c["vgx_last_error"]().decode(errors="replace")


def version():
    return _c["vgx_version"]().decode()


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------
def _stream(stream=None):
    import torch
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dptr(t, dtype=None, numel=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return C.c_void_p(t.data_ptr())


def _hptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# ---------------------------------------------------------------------------
# PDF
# ---------------------------------------------------------------------------
def pdf_create(x_knots, q2_knots, xf, stream=None):
    """x_knots (n_x,), q2_knots list of per-subgrid arrays, xf list of
    (n_flav, n_q[s], n_x) arrays (host, FP64).  Returns an opaque handle."""
    x = np.ascontiguousarray(x_knots, dtype=np.float64)
    nq = np.ascontiguousarray([len(q) for q in q2_knots], dtype=np.int32)
    q2 = np.ascontiguousarray(np.concatenate([np.asarray(q, dtype=np.float64) for q in q2_knots]))
    vals = np.ascontiguousarray(np.concatenate([np.asarray(v, dtype=np.float64).ravel() for v in xf]))
    n_flav = int(np.asarray(xf[0]).shape[0])
    d = PdfDesc(len(x), len(nq), n_flav, _hptr(x, _f64), _hptr(nq, _i32), _hptr(q2, _f64), _hptr(vals, _f64))
    h = _vp()
    _check(_c["pdf_create"](C.byref(d), _stream(stream), C.byref(h)), "pdf_create")
    return h


def pdf_create_set(x_knots, q2_knots, xf_members, stream=None):
    """A PDF set: xf_members is a list (one per member) of xf lists as for
    pdf_create; all members share the knots."""
    x = np.ascontiguousarray(x_knots, dtype=np.float64)
    nq = np.ascontiguousarray([len(q) for q in q2_knots], dtype=np.int32)
    q2 = np.ascontiguousarray(np.concatenate([np.asarray(q, dtype=np.float64) for q in q2_knots]))
    vals = np.ascontiguousarray(np.concatenate([np.asarray(v, dtype=np.float64).ravel()
                                                for member in xf_members for v in member]))
    n_flav = int(np.asarray(xf_members[0][0]).shape[0])
    d = PdfDesc(len(x), len(nq), n_flav, _hptr(x, _f64), _hptr(nq, _i32), _hptr(q2, _f64), _hptr(vals, _f64))
    h = _vp()
    _check(_c["pdf_create_set"](C.byref(d), len(xf_members), _stream(stream), C.byref(h)), "pdf_create_set")
    return h


def pdf_shape(pdf):
    nf, nm = _i32(), _i32()
    _check(_c["pdf_shape"](pdf, C.byref(nf), C.byref(nm)), "pdf_shape")
    return int(nf.value), int(nm.value)


def pdf_interp(pdf, x, q2, out, out_dtype=None, stream=None):
    import torch
    n = x.numel()
    if out_dtype is None:
        out_dtype = F64 if out.dtype == torch.float64 else F32
    want = torch.float64 if out_dtype == F64 else torch.float32
    nf, _ = pdf_shape(pdf)
    _check(_c["pdf_interp"](pdf, n, _dptr(x, torch.float64, n, "x"), _dptr(q2, torch.float64, n, "q2"), out_dtype,
                            _dptr(out, want, nf * n, "out"), _stream(stream)), "pdf_interp")
    return out


def pdf_interp_members(pdf, x, q2, out, out_dtype=None, stream=None):
    """out: CUDA (n_members, n_flav, n)."""
    import torch
    n = x.numel()
    if out_dtype is None:
        out_dtype = F64 if out.dtype == torch.float64 else F32
    want = torch.float64 if out_dtype == F64 else torch.float32
    nf, nm = pdf_shape(pdf)
    _check(_c["pdf_interp_members"](pdf, n, _dptr(x, torch.float64, n, "x"), _dptr(q2, torch.float64, n, "q2"),
                                    out_dtype, _dptr(out, want, nm * nf * n, "out"), _stream(stream)),
           "pdf_interp_members")
    return out


def pdf_out_of_range(pdf, stream=None):
    c = _i64()
    st = _c["pdf_out_of_range"](pdf, _stream(stream), C.byref(c))
    if st not in (VGX_OK, VGX_ERANGE):
        _check(st, "pdf_out_of_range")
    return int(c.value)


def pdf_bounds(pdf):
    v = [_f64() for _ in range(4)]
    _check(_c["pdf_bounds"](pdf, *[C.byref(t) for t in v]), "pdf_bounds")
    return tuple(t.value for t in v)


def pdf_set_extrapolation(pdf, mode):
    _check(_c["pdf_set_extrapolation"](pdf, int(mode)), "pdf_set_extrapolation")


def pdf_set_alphas(pdf, q2_knots, alphas, stream=None):
    """q2_knots: host (n,) ascending, a repeated knot starting a new subgrid
    (or a list of per-subgrid arrays, concatenated here); alphas likewise."""
    if isinstance(q2_knots, (list, tuple)):
        q2_knots = np.concatenate([np.asarray(q, dtype=np.float64) for q in q2_knots])
        alphas = np.concatenate([np.asarray(a, dtype=np.float64) for a in alphas])
    q = np.ascontiguousarray(q2_knots, dtype=np.float64)
    a = np.ascontiguousarray(alphas, dtype=np.float64)
    if q.shape != a.shape:
        raise ValueError("q2_knots and alphas differ in length")
    _check(_c["pdf_set_alphas"](pdf, q.size, _hptr(q, _f64), _hptr(a, _f64), _stream(stream)), "pdf_set_alphas")


def pdf_alphas(pdf, q2, out, stream=None):
    import torch
    n = q2.numel()
    _check(_c["pdf_alphas"](pdf, n, _dptr(q2, torch.float64, n, "q2"), _dptr(out, torch.float64, n, "out"),
                            _stream(stream)), "pdf_alphas")
    return out


def pdf_destroy(pdf):
    _c["pdf_destroy"](pdf)


# ---------------------------------------------------------------------------
# Event generation
# ---------------------------------------------------------------------------
def rambo_generate(masses, sqrt_s, seed, stream_id, iteration, first, mom, w, stream=None):
    """masses: host (n,); mom: CUDA float64 (4, n, N); w: CUDA float64 (N,)."""
    import torch
    m = np.ascontiguousarray(masses, dtype=np.float64)
    n_ev = w.numel()
    _check(_c["rambo_generate"](m.size, _hptr(m, _f64), float(sqrt_s), int(seed), int(stream_id), int(iteration),
                                int(first), n_ev, _dptr(mom, torch.float64, 4 * m.size * n_ev, "mom"),
                                _dptr(w, torch.float64, n_ev, "w"), _stream(stream)), "rambo_generate")
    return mom, w


def lhe_open(path, beam_id=(2212, 2212), beam_energy=(6500.0, 6500.0), pdf_group=(0, 0), pdf_set=(-1, -1),
             weight_mode=3, xsec=0.0, xsec_err=0.0, xmax=1.0, proc_id=1):
    ini = LheInit((_i32 * 2)(*beam_id), (_f64 * 2)(*beam_energy), (_i32 * 2)(*pdf_group), (_i32 * 2)(*pdf_set),
                  weight_mode, xsec, xsec_err, xmax, proc_id)
    h = _vp()
    _check(_c["lhe_open"](os.fsencode(path), C.byref(ini), C.byref(h)), "lhe_open")
    return h


def _lhe_meta(pdg_in, pdg_out, masses, sqrt_s, weight, scale, aqed, aqcd, proc_id):
    pi = np.ascontiguousarray(pdg_in, dtype=np.int32)
    po = np.ascontiguousarray(pdg_out, dtype=np.int32)
    m = np.ascontiguousarray(masses, dtype=np.float64)
    if pi.size != 2 or po.size != m.size:
        raise ValueError("pdg_in needs 2 codes and pdg_out one per mass")
    return pi, po, m, LheEventInfo(sqrt_s, weight, scale, aqed, aqcd, proc_id)


def lhe_write_events(h, mom, idx, n_kept, pdg_in, pdg_out, masses, sqrt_s, weight=1.0, scale=0.0, aqed=0.0,
                     aqcd=0.0, proc_id=1, stream=None):
    """Queue events idx[:n_kept] (idx None: 0..n_kept-1) of a rambo_generate
    output mom (4, n, N)."""
    import torch
    pi, po, m, info = _lhe_meta(pdg_in, pdg_out, masses, sqrt_s, weight, scale, aqed, aqcd, proc_id)
    n_total = mom.shape[2]
    _check(_c["lhe_write_events"](h, po.size, _hptr(pi, _i32), _hptr(po, _i32), _hptr(m, _f64), C.byref(info),
                                  n_total, _dptr(mom, torch.float64, 4 * po.size * n_total, "mom"),
                                  _dptr(idx, torch.int64, n_kept, "idx"), int(n_kept), _stream(stream)),
           "lhe_write_events")


def lhe_write_events_host(h, mom, pdg_in, pdg_out, masses, sqrt_s, weight=1.0, scale=0.0, aqed=0.0, aqcd=0.0,
                          proc_id=1):
    """Queue events from host memory: mom (N, n, 4) (E, px, py, pz)."""
    pi, po, m, info = _lhe_meta(pdg_in, pdg_out, masses, sqrt_s, weight, scale, aqed, aqcd, proc_id)
    a = np.ascontiguousarray(mom, dtype=np.float64)
    if a.ndim != 3 or a.shape[1] != po.size or a.shape[2] != 4:
        raise ValueError("mom must be (N, n_part, 4)")
    _check(_c["lhe_write_events_host"](h, po.size, _hptr(pi, _i32), _hptr(po, _i32), _hptr(m, _f64), C.byref(info),
                                       a.shape[0], _hptr(a, _f64)), "lhe_write_events_host")


def lhe_flush(h):
    n = _i64()
    _check(_c["lhe_flush"](h, C.byref(n)), "lhe_flush")
    return int(n.value)


def lhe_close(h):
    _check(_c["lhe_close"](h), "lhe_close")


class LheWriter:
    """Context manager over lhe_open / lhe_write_events / lhe_close; the
    library's own thread formats and writes the records."""

    def __init__(self, path, **init):
        self._h = lhe_open(path, **init)

    def write(self, mom, idx, n_kept, *args, **kw):
        lhe_write_events(self._h, mom, idx, n_kept, *args, **kw)

    def write_host(self, mom, *args, **kw):
        lhe_write_events_host(self._h, mom, *args, **kw)

    def flush(self):
        return lhe_flush(self._h)

    def close(self):
        if self._h is not None:
            h, self._h = self._h, None
            lhe_close(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False


def unweight(w, seed, stream_id, iteration, idx, w_max=0.0, stream=None):
    """Kept event indices (ascending) into idx[:n_kept]; returns (n_kept, w_max_used)."""
    import torch
    n = w.numel()
    k, wm = _i64(), _f64()
    _check(_c["unweight"](n, _dptr(w, torch.float64, n, "w"), float(w_max), int(seed), int(stream_id),
                          int(iteration), _dptr(idx, torch.int64, n, "idx"), C.byref(k), C.byref(wm),
                          _stream(stream)), "unweight")
    return int(k.value), float(wm.value)


UNWEIGHT_NOALLOC_MAX = 65945600


def unweight_noalloc(w, seed, stream_id, iteration, idx, w_max=0.0, stream=None):
    """unweight() without any device allocation (fixed scratch array); n up to
    UNWEIGHT_NOALLOC_MAX."""
    import torch
    n = w.numel()
    k, wm = _i64(), _f64()
    _check(_c["unweight_noalloc"](n, _dptr(w, torch.float64, n, "w"), float(w_max), int(seed), int(stream_id),
                                  int(iteration), _dptr(idx, torch.int64, n, "idx"), C.byref(k), C.byref(wm),
                                  _stream(stream)), "unweight_noalloc")
    return int(k.value), float(wm.value)


# ---------------------------------------------------------------------------
# VEGAS
# ---------------------------------------------------------------------------
def vegas_create(kind, dim, n_bins, alpha, seed, stream_id=0, prec=F64, params=(), pdf=None, stream=None):
    p = np.ascontiguousarray(params, dtype=np.float64)
    cfg = VegasCfg(kind, dim, n_bins, alpha, seed, stream_id, prec, _hptr(p, _f64) if p.size else None, p.size,
                   pdf)
    h = _vp()
    _check(_c["vegas_create"](C.byref(cfg), _stream(stream), C.byref(h)), "vegas_create")
    return h


def vegas_iterate(v, n, iteration, allow_numeric=False):
    r = IterResult()
    st = _c["vegas_iterate"](v, n, iteration, C.byref(r))
    if not (allow_numeric and st == VGX_ENUMERIC):
        _check(st, "vegas_iterate")
    return r.as_dict()


def vegas_iterate_async(v, n, iteration):
    _check(_c["vegas_iterate_async"](v, n, iteration), "vegas_iterate_async")


def vegas_refine(v):
    _check(_c["vegas_refine"](v), "vegas_refine")


def vegas_result(v):
    m, s, c, k = _f64(), _f64(), _f64(), _i32()
    _check(_c["vegas_result"](v, C.byref(m), C.byref(s), C.byref(c), C.byref(k)), "vegas_result")
    return dict(mean=m.value, sigma=s.value, chi2_dof=c.value, n_used=k.value)


def vegas_results(v, cap=4096):
    arr = (IterResult * cap)()
    cnt = _i32()
    _check(_c["vegas_results"](v, arr, cap, C.byref(cnt)), "vegas_results")
    return [arr[k].as_dict() for k in range(min(cnt.value, cap))]


def vegas_reset_results(v):
    _check(_c["vegas_reset_results"](v), "vegas_reset_results")


def vegas_get_grid(v, dim, n_bins):
    e = np.empty((dim, n_bins + 1), dtype=np.float64)
    _check(_c["vegas_get_grid"](v, _hptr(e, _f64)), "vegas_get_grid")
    return e


def vegas_set_grid(v, edges):
    e = np.ascontiguousarray(edges, dtype=np.float64)
    _check(_c["vegas_set_grid"](v, _hptr(e, _f64)), "vegas_set_grid")


def vegas_get_hist(v, dim, n_bins):
    h = np.empty((dim, n_bins), dtype=np.float64)
    _check(_c["vegas_get_hist"](v, _hptr(h, _f64)), "vegas_get_hist")
    return h


def vegas_shape(v):
    d, nb = _i32(), _i32()
    _check(_c["vegas_shape"](v, C.byref(d), C.byref(nb)), "vegas_shape")
    return int(d.value), int(nb.value)


def vegas_sample(v, first, n, iteration, u=None, g=None):
    import torch
    dim, _ = vegas_shape(v)
    _check(_c["vegas_sample"](v, first, n, iteration, _dptr(u, torch.float64, dim * n if u is not None else None, "u"),
                              _dptr(g, torch.float64, n if g is not None else None, "g")), "vegas_sample")


def vegas_iterate_points(v, y, logq=None, allow_numeric=False, allow_fallback=False):
    """Estimate from caller points; with allow_fallback a proposal judged
    worse than plain VEGAS (VGX_EFALLBACK) returns its result with
    fallback=True instead of raising."""
    import torch
    n = y.shape[-1]
    r = IterResult()
    dim, _ = vegas_shape(v)
    st = _c["vegas_iterate_points"](v, n, _dptr(y, torch.float64, dim * n, "y"),
                                    _dptr(logq, torch.float64, n if logq is not None else None, "logq"),
                                    C.byref(r))
    if not ((allow_numeric and st == VGX_ENUMERIC) or (allow_fallback and st == VGX_EFALLBACK)):
        _check(st, "vegas_iterate_points")
    d = r.as_dict()
    d["fallback"] = st == VGX_EFALLBACK
    return d


def vegas_stream(v):
    return _c["vegas_stream"](v)


def vegas_set_timing(v, enable=True, every=1):
    """Time one fused kernel in `every` (enable=False: off)."""
    _check(_c["vegas_set_timing"](v, int(every) if enable else 0), "vegas_set_timing")


def vegas_kernel_time(v):
    ms, k = _f64(), _i64()
    _check(_c["vegas_kernel_time"](v, C.byref(ms), C.byref(k)), "vegas_kernel_time")
    return ms.value, k.value


def vegas_destroy(v):
    _c["vegas_destroy"](v)


# ---------------------------------------------------------------------------
# Batched integration
# ---------------------------------------------------------------------------
def batch_create(ctxs, n_samples, tile=0, block=0, stream=None):
    arr = (_vp * len(ctxs))(*[c.value if isinstance(c, _vp) else c for c in ctxs])
    ns = np.ascontiguousarray(n_samples, dtype=np.int64)
    h = _vp()
    _check(_c["batch_create"](arr, len(ctxs), _hptr(ns, _i64), tile, block, _stream(stream), C.byref(h)),
           "batch_create")
    return h


def batch_iterate(b, iteration, count):
    arr = (IterResult * count)()
    _check(_c["batch_iterate"](b, iteration, arr), "batch_iterate")
    return [arr[k].as_dict() for k in range(count)]


def batch_config(b):
    t, bl = _i32(), _i32()
    _check(_c["batch_config"](b, C.byref(t), C.byref(bl)), "batch_config")
    return t.value, bl.value


def batch_destroy(b):
    _c["batch_destroy"](b)


# ---------------------------------------------------------------------------
# Flow
# ---------------------------------------------------------------------------
def flow_num_params(dim, n_layers=4, n_bins=32, hidden=64):
    return int(_c["flow_num_params"](dim, n_layers, n_bins, hidden))


def flow_param_layout(dim, n_layers=4, n_bins=32, hidden=64):
    """[(kind, fan_in, size)] per parameter segment; kind "w", "b" or "z"
    (output layer), in the flat parameter order."""
    cap = 6 * n_layers
    kind = np.zeros(cap, dtype=np.int32)
    fan = np.zeros(cap, dtype=np.int32)
    size = np.zeros(cap, dtype=np.int64)
    n = _i32()
    _check(_c["flow_param_layout"](dim, n_layers, n_bins, hidden, _hptr(kind, _i32), _hptr(fan, _i32),
                                   _hptr(size, _i64), cap, C.byref(n)), "flow_param_layout")
    names = {0: "w", 1: "b", 2: "z"}
    return [(names[int(kind[k])], int(fan[k]), int(size[k])) for k in range(n.value)]


def flow_create(dim, params, n_layers=4, n_bins=32, hidden=64, stream=None):
    p = np.ascontiguousarray(params, dtype=np.float32)
    h = _vp()
    _check(_c["flow_create"](dim, n_layers, n_bins, hidden, _hptr(p, _f32), p.size, _stream(stream), C.byref(h)),
           "flow_create")
    return h


def flow_shape(f):
    d, npar = _i32(), _i64()
    _check(_c["flow_shape"](f, C.byref(d), C.byref(npar)), "flow_shape")
    return int(d.value), int(npar.value)


def flow_sample(f, n, seed, stream_id, iteration, y, logq, stream=None):
    import torch
    dim, _ = flow_shape(f)
    _check(_c["flow_sample"](f, n, seed, stream_id, iteration, _dptr(y, torch.float64, dim * n, "y"),
                             _dptr(logq, torch.float64, n, "logq"), _stream(stream)), "flow_sample")


def flow_vegas_iterate(f, v, n, seed, stream_id, iteration, allow_numeric=False, allow_fallback=False):
    """n points from the flow weighted into the VEGAS context's estimate in
    one pass (the points flow_sample would draw; no points in memory)."""
    r = IterResult()
    st = _c["flow_vegas_iterate"](f, v, n, seed, stream_id, iteration, C.byref(r))
    if not ((allow_numeric and st == VGX_ENUMERIC) or (allow_fallback and st == VGX_EFALLBACK)):
        _check(st, "flow_vegas_iterate")
    d = r.as_dict()
    d["fallback"] = st == VGX_EFALLBACK
    return d


def flow_density(f, y, logq, u=None, stream=None):
    import torch
    n = y.shape[-1]
    dim, _ = flow_shape(f)
    _check(_c["flow_density"](f, n, _dptr(y, torch.float64, dim * n, "y"),
                              _dptr(u, torch.float64, dim * n if u is not None else None, "u"),
                              _dptr(logq, torch.float64, n, "logq"), _stream(stream)), "flow_density")


def flow_loss_grad(f, y, g, n_params=None):
    import torch
    n = y.shape[-1]
    loss = _f64()
    grad = np.empty(n_params, dtype=np.float32) if n_params else None
    dim, _ = flow_shape(f)
    _check(_c["flow_loss_grad"](f, n, _dptr(y, torch.float64, dim * n, "y"), _dptr(g, torch.float64, n, "g"),
                                C.byref(loss), _hptr(grad, _f32) if grad is not None else None), "flow_loss_grad")
    return loss.value, grad


def flow_train_step(f, y, g, lr, sync=True, allow_fallback=False):
    import torch
    n = y.shape[-1]
    loss = _f64()
    dim, _ = flow_shape(f)
    st = _c["flow_train_step"](f, n, _dptr(y, torch.float64, dim * n, "y"), _dptr(g, torch.float64, n, "g"), lr,
                               C.byref(loss) if sync else None)
    if not (allow_fallback and st == VGX_EFALLBACK):
        _check(st, "flow_train_step")
    return loss.value if sync else None


def flow_adam(f, grad, lr):
    import torch
    _, n_par = flow_shape(f)
    _check(_c["flow_adam"](f, _dptr(grad, torch.float32, n_par, "grad"), lr), "flow_adam")


def flow_get_params(f, n_params):
    p = np.empty(n_params, dtype=np.float32)
    n = _i64()
    _check(_c["flow_get_params"](f, _hptr(p, _f32), n_params, C.byref(n)), "flow_get_params")
    return p[:n.value]


def flow_set_params(f, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(_c["flow_set_params"](f, _hptr(p, _f32), p.size), "flow_set_params")


def flow_set_operands(f, operands):
    """OPERANDS_BF16 (the product path) or OPERANDS_F32 (validation mode)."""
    _check(_c["flow_set_operands"](f, int(operands)), "flow_set_operands")


def flow_destroy(f):
    _c["flow_destroy"](f)
