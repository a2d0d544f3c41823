"""ctypes binding of libmisdc.so (argument marshalling only).

Every function of the C ABI (include/misdc.h) is exposed under the same name;
torch tensors are passed as device pointers and torch streams as hipStream_t.
No arithmetic of the method happens here: every step runs in the library's
HIP kernels.  Importing this module raises if the library has not been
built; nothing falls back to another implementation.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmisdc.so")

MISDC_OK = 0
MISDC_EINVAL = -1
MISDC_ENOMEM = -2
MISDC_EDEVICE = -3
MISDC_ENOTCONV = -4
MISDC_EUNSUPPORTED = -5
MISDC_ESTATE = -6
SCHEME = {"misdc": 0, "misdcq": 1, "cisdcq": 2, "imexq": 3}
QE = {"cumulative": 0, "literal": 1}
QI = {"lu": 0, "be": 1}

EXPORTED = [
    "misdc_last_error", "misdc_version", "misdc_sdc_tables", "misdc_mech_create",
    "misdc_mech_destroy", "misdc_mech_species", "misdc_enthalpy", "misdc_temperature",
    "misdc_reaction_source", "misdc_reaction_solve_batch", "misdc_grid_create",
    "misdc_grid_create_ensemble", "misdc_grid_destroy", "misdc_grid_cells",
    "misdc_transport_operators", "misdc_diffusion_solve", "misdc_opts_default",
    "misdc_integ_create", "misdc_integ_destroy", "misdc_step", "misdc_step_begin",
    "misdc_sweep", "misdc_step_end", "misdc_get_stats",
    "misdc_get_newton_histogram", "misdc_reset_profile", "misdc_autotune", "misdc_get_tune", "misdc_set_tune",
    "misdc_mlp_create", "misdc_mlp_destroy", "misdc_mlp_param_count", "misdc_mlp_set_params",
    "misdc_mlp_get_params", "misdc_mlp_set_normalization", "misdc_mlp_forward",
    "misdc_mlp_gradients", "misdc_mlp_adam_step", "misdc_mlp_train", "misdc_mlp_features",
    "misdc_mlp_targets", "misdc_reaction_guess_mlp", "misdc_integ_set_guess",
    "misdc_integ_record", "misdc_integ_recorded", "misdc_set_streams", "misdc_mlp_prepare_training",
    "misdc_diffusion_solve_noalloc", "misdc_mech_specialized", "misdc_mech_generate",
]
MLP_PRECISION = {"bf16": 0, "fp32": 1}
NEWTON_KERNEL = {"auto": 0, "thread": 1, "wave": 2, "specialized": 3}


class MisdcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"misdc error {code}: {msg}")
        self.code = code


class misdc_mech_desc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32), ("bath", C.c_int32),
                ("W", C.c_void_p), ("react", C.c_void_p), ("prod", C.c_void_p),
                ("A", C.c_void_p), ("beta", C.c_void_p), ("Ea", C.c_void_p),
                ("cp", C.c_void_p), ("hf", C.c_void_p), ("s0", C.c_void_p), ("D0", C.c_void_p),
                ("alpha0", C.c_double), ("rho0", C.c_double), ("p_atm", C.c_double),
                ("R_u", C.c_double), ("R_c", C.c_double)]


class misdc_newton_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("dtau0", C.c_double),
                ("dtau_max", C.c_double), ("neg_slack", C.c_double), ("kernel", C.c_int32),
                ("lu", C.c_int32)]


class misdc_opts(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_sweeps", C.c_int32), ("nu", C.c_int32),
                ("scheme", C.c_int32), ("qe_mode", C.c_int32), ("serialize", C.c_int32),
                ("newton", misdc_newton_opts), ("cg_rtol", C.c_double), ("cg_maxit", C.c_int32),
                ("profile", C.c_int32), ("use_graph", C.c_int32), ("nu_tol", C.c_double),
                ("pipeline", C.c_int32), ("imexq_tol", C.c_double), ("imexq_maxit", C.c_int32),
                ("imexq_krylov_rtol", C.c_double), ("imexq_krylov_maxit", C.c_int32)]


class misdc_tune(C.Structure):
    _fields_ = [("cg_variant", C.c_int32), ("cg_blocks", C.c_int32), ("cyclic", C.c_int32),
                ("serialize", C.c_int32), ("cu_split", C.c_int32),
                ("stagger", C.c_int32), ("step_ms", C.c_double), ("fused", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class misdc_stats(C.Structure):
    _fields_ = [("newton_solves", C.c_int64), ("newton_iters", C.c_int64),
                ("newton_max", C.c_int32), ("newton_failed", C.c_int64),
                ("cg_solves", C.c_int64), ("cg_iters", C.c_int64), ("cg_max", C.c_int32),
                ("cg_failed", C.c_int32), ("n_sweeps", C.c_int32),
                ("sweep_increment", C.c_double * 64), ("diffusion_kernel_ms", C.c_double),
                ("diffusion_kernel_launches", C.c_int64), ("newton_kernel_ms", C.c_double),
                ("newton_kernel_launches", C.c_int64), ("newton_lu_solves", C.c_int64),
                ("newton_lu_fallbacks", C.c_int64), ("newton_guess_learned", C.c_int64),
                ("nested_passes", C.c_int32 * 64), ("newton_pivot_retries", C.c_int64),
                ("imexq_solves", C.c_int64), ("imexq_newton_iters", C.c_int64),
                ("imexq_failed", C.c_int64), ("imexq_krylov_iters", C.c_int64),
                ("imexq_krylov_max", C.c_int64), ("imexq_krylov_failed", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_
             if k not in ("sweep_increment", "nested_passes")}
        d["sweep_increment"] = list(self.sweep_increment[:self.n_sweeps])
        d["nested_passes"] = list(self.nested_passes[:self.n_sweeps])
        return d


def load(path=LIB_PATH):
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run paper_1801_01201_amd.build.build()")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "misdc_last_error": (C.c_char_p, []),
        "misdc_version": (C.c_char_p, []),
        "misdc_sdc_tables": (C.c_int, [C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp]),
        "misdc_mech_create": (C.c_int, [C.POINTER(misdc_mech_desc), C.POINTER(vp)]),
        "misdc_mech_destroy": (C.c_int, [vp]),
        "misdc_mech_species": (C.c_int, [vp, C.POINTER(i32)]),
        "misdc_mech_specialized": (C.c_int, [vp, C.POINTER(i32), C.POINTER(C.c_char_p)]),
        "misdc_mech_generate": (C.c_int, [C.POINTER(misdc_mech_desc), C.c_int, C.c_char_p,
                                          C.POINTER(C.c_size_t)]),
        "misdc_enthalpy": (C.c_int, [vp, i64, vp, vp, vp, vp]),
        "misdc_temperature": (C.c_int, [vp, i64, vp, vp, vp, vp]),
        "misdc_reaction_source": (C.c_int, [vp, i64, vp, vp, vp, vp]),
        "misdc_reaction_solve_batch": (C.c_int, [vp, i64, vp, vp, vp, vp, vp, vp, vp,
                                                 C.POINTER(misdc_newton_opts), vp]),
        "misdc_grid_create": (C.c_int, [C.c_int, vp, vp, vp, C.POINTER(vp)]),
        "misdc_grid_create_ensemble": (C.c_int, [C.c_int, vp, vp, vp, C.POINTER(vp)]),
        "misdc_grid_destroy": (C.c_int, [vp]),
        "misdc_grid_cells": (C.c_int, [vp, C.POINTER(i64)]),
        "misdc_transport_operators": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "misdc_diffusion_solve": (C.c_int, [vp, vp, dbl, vp, vp, vp, C.c_int, dbl, C.c_int,
                                            vp, vp]),
        "misdc_diffusion_solve_noalloc": (C.c_int, [vp, vp, dbl, vp, vp, vp, C.c_int, dbl,
                                                    C.c_int, vp, vp]),
        "misdc_opts_default": (None, [C.POINTER(misdc_opts)]),
        "misdc_integ_create": (C.c_int, [vp, vp, C.POINTER(misdc_opts), C.POINTER(vp)]),
        "misdc_integ_destroy": (C.c_int, [vp]),
        "misdc_step": (C.c_int, [vp, vp, dbl, vp, vp]),
        "misdc_get_stats": (C.c_int, [vp, C.POINTER(misdc_stats)]),
        "misdc_get_newton_histogram": (C.c_int, [vp, C.c_int, C.POINTER(C.c_int64)]),
        "misdc_step_begin": (C.c_int, [vp, vp, C.c_double, vp, vp]),
        "misdc_sweep": (C.c_int, [vp, vp]),
        "misdc_step_end": (C.c_int, [vp, vp]),
        "misdc_reset_profile": (C.c_int, [vp]),
        "misdc_autotune": (C.c_int, [vp, vp, dbl, vp, C.c_int, C.POINTER(misdc_tune), vp]),
        "misdc_get_tune": (C.c_int, [vp, C.POINTER(misdc_tune)]),
        "misdc_set_tune": (C.c_int, [vp, C.POINTER(misdc_tune)]),
        "misdc_mlp_create": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(vp)]),
        "misdc_mlp_destroy": (C.c_int, [vp]),
        "misdc_mlp_param_count": (C.c_int, [vp, C.POINTER(i64)]),
        "misdc_mlp_set_params": (C.c_int, [vp, vp]),
        "misdc_mlp_get_params": (C.c_int, [vp, vp]),
        "misdc_mlp_set_normalization": (C.c_int, [vp, vp, vp, vp]),
        "misdc_mlp_forward": (C.c_int, [vp, i64, vp, vp, vp]),
        "misdc_mlp_gradients": (C.c_int, [vp, i64, vp, vp, vp, vp, vp]),
        "misdc_mlp_adam_step": (C.c_int, [vp, vp, C.c_float, C.c_float, C.c_float, C.c_float, vp]),
        "misdc_mlp_train": (C.c_int, [vp, i64, vp, vp, i64, C.c_int, C.c_float, vp, vp]),
        "misdc_mlp_features": (C.c_int, [vp, vp, i64, vp, vp, vp, vp, vp]),
        "misdc_mlp_targets": (C.c_int, [vp, vp, i64, vp, vp, vp, vp, vp]),
        "misdc_reaction_guess_mlp": (C.c_int, [vp, vp, i64, vp, vp, vp, vp, vp, vp]),
        "misdc_integ_set_guess": (C.c_int, [vp, vp, C.c_int]),
        "misdc_integ_record": (C.c_int, [vp, vp, i64]),
        "misdc_integ_recorded": (C.c_int, [vp, C.POINTER(i64)]),
        "misdc_set_streams": (C.c_int, [vp, vp, vp]),
        "misdc_mlp_prepare_training": (C.c_int, [vp, vp, i64, vp, vp, vp, vp, C.c_uint64, vp, vp,
                                                 vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


def check(code):
    if code != MISDC_OK:
        raise MisdcError(code, lib().misdc_last_error().decode())
    return code


def _ptr(t):
    """Device (or host numpy) pointer of a tensor/array; None stays NULL."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------------------
# C ABI, same names
# ---------------------------------------------------------------------------
def misdc_version():
    return lib().misdc_version().decode()


def misdc_sdc_tables(n_nodes, qi="lu", qe="cumulative"):
    M = n_nodes - 1
    out = dict(tau=np.zeros(M + 1), Q=np.zeros((M, M + 1)), QI=np.zeros((M, M)),
               QE=np.zeros((M, M)), S=np.zeros((M, M + 1)))
    check(lib().misdc_sdc_tables(n_nodes, QI[qi], QE[qe], _ptr(out["tau"]), _ptr(out["Q"]),
                                 _ptr(out["QI"]), _ptr(out["QE"]), _ptr(out["S"])))
    return out


def _mech_desc(mech, keep):
    """misdc_mech_desc of a mechanism dict in the generator's format (host
    arrays kept alive in ``keep``)."""

    def arr(key, dtype):
        a = np.ascontiguousarray(np.asarray(mech[key], dtype=dtype))
        keep[key] = a
        return a.ctypes.data

    d = misdc_mech_desc()
    d.n_species = int(mech["N"])
    d.n_reactions = int(mech["R"])
    d.bath = int(mech["bath"])
    d.W = arr("W", np.float64)
    d.react = arr("react", np.int32)
    d.prod = arr("prod", np.int32)
    for k in ("A", "beta", "Ea", "cp", "hf", "s0", "D0"):
        setattr(d, k, arr(k, np.float64))
    d.alpha0 = float(mech["alpha0"])
    d.rho0 = float(mech["rho0"])
    d.p_atm = float(mech["p_atm"])
    d.R_u = float(mech["R_u"])
    d.R_c = float(mech["R_c"])
    return d


def misdc_mech_create(mech):
    """mech: dict in the generator's format (host arrays)."""
    keep = {}
    d = _mech_desc(mech, keep)
    h = C.c_void_p()
    check(lib().misdc_mech_create(C.byref(d), C.byref(h)))
    return h.value


def misdc_mech_specialized(h):
    """(available, status message) of the reaction solve generated for a
    mechanism."""
    av = C.c_int32()
    msg = C.c_char_p()
    check(lib().misdc_mech_specialized(h, C.byref(av), C.byref(msg)))
    return bool(av.value), msg.value.decode()


def misdc_mech_generate(mech, compile=False):
    """Source text generated for a mechanism (host only); with compile, also
    compiled for the device by hiprtc."""
    keep = {}
    d = _mech_desc(mech, keep)
    n = C.c_size_t(0)
    check(lib().misdc_mech_generate(C.byref(d), int(bool(compile)), None, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    check(lib().misdc_mech_generate(C.byref(d), 0, buf, C.byref(n)))
    return buf.value.decode()


def misdc_mech_destroy(h):
    check(lib().misdc_mech_destroy(h))


def misdc_enthalpy(mech, n, Y, T, h, stream=None):
    check(lib().misdc_enthalpy(mech, n, _ptr(Y), _ptr(T), _ptr(h), _stream(stream)))


def misdc_temperature(mech, n, Y, h, T, stream=None):
    check(lib().misdc_temperature(mech, n, _ptr(Y), _ptr(h), _ptr(T), _stream(stream)))


def misdc_reaction_source(mech, n, Y, h, FR, stream=None):
    check(lib().misdc_reaction_source(mech, n, _ptr(Y), _ptr(h), _ptr(FR), _stream(stream)))


LU = {"fp64": 0, "fp32_mfma": 1}


def newton_opts(tol=0.0, maxit=0, dtau0=0.0, dtau_max=0.0, neg_slack=0.0, kernel="auto",
                lu="fp64"):
    return misdc_newton_opts(tol, maxit, dtau0, dtau_max, neg_slack, NEWTON_KERNEL[kernel],
                             LU[lu])


def misdc_reaction_solve_batch(mech, n, bY, h, c, Y, T_out=None, FR_out=None, iters=None,
                               opts=None, stream=None):
    o = opts if opts is not None else newton_opts()
    check(lib().misdc_reaction_solve_batch(mech, n, _ptr(bY), _ptr(h), _ptr(c), _ptr(Y),
                                           _ptr(T_out), _ptr(FR_out), _ptr(iters), C.byref(o),
                                           _stream(stream)))


def misdc_grid_create(dim, n, dx, u):
    nn = np.asarray(n, dtype=np.int64)
    dd = np.asarray(dx, dtype=np.float64)
    uu = np.asarray(u, dtype=np.float64)
    h = C.c_void_p()
    check(lib().misdc_grid_create(dim, _ptr(nn), _ptr(dd), _ptr(uu), C.byref(h)))
    return h.value


def misdc_grid_create_ensemble(lengths, dx, u):
    ll = np.ascontiguousarray(lengths, dtype=np.int64)
    dd = np.ascontiguousarray(dx, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    h = C.c_void_p()
    check(lib().misdc_grid_create_ensemble(len(ll), _ptr(ll), _ptr(dd), _ptr(uu), C.byref(h)))
    return h.value


def misdc_grid_destroy(h):
    check(lib().misdc_grid_destroy(h))


def misdc_transport_operators(mech, grid, state, FA, FD, stream=None):
    check(lib().misdc_transport_operators(mech, grid, _ptr(state), _ptr(FA), _ptr(FD),
                                          _stream(stream)))


def misdc_diffusion_solve(mech, grid, c, T_lag, rhs, y, guess_in_y=False, rtol=0.0, maxit=0,
                          iters=None, stream=None):
    check(lib().misdc_diffusion_solve(mech, grid, float(c), _ptr(T_lag), _ptr(rhs), _ptr(y),
                                      int(bool(guess_in_y)), float(rtol), int(maxit),
                                      _ptr(iters), _stream(stream)))


def misdc_opts_default():
    o = misdc_opts()
    lib().misdc_opts_default(C.byref(o))
    return o


def misdc_integ_create(mech, grid, opts):
    h = C.c_void_p()
    check(lib().misdc_integ_create(mech, grid, C.byref(opts), C.byref(h)))
    return h.value


def misdc_integ_destroy(h):
    check(lib().misdc_integ_destroy(h))


def misdc_step(integ, state, dt, dt_per_flame=None, stream=None):
    check(lib().misdc_step(integ, _ptr(state), float(dt), _ptr(dt_per_flame), _stream(stream)))


def misdc_step_begin(integ, state, dt, dt_per_flame=None, stream=None):
    check(lib().misdc_step_begin(integ, _ptr(state), float(dt), _ptr(dt_per_flame),
                                 _stream(stream)))


def misdc_sweep(integ, stream=None):
    check(lib().misdc_sweep(integ, _stream(stream)))


def misdc_step_end(integ, stream=None):
    check(lib().misdc_step_end(integ, _stream(stream)))


def misdc_set_streams(integ, diffusion_stream=None, reaction_stream=None):
    """Run the diffusion and reaction tasks on the caller's streams (torch
    streams or raw hipStream_t ints); None selects the integrator's own."""
    def raw(s):
        if s is None:
            return None
        return s if isinstance(s, int) else s.cuda_stream
    check(lib().misdc_set_streams(integ, raw(diffusion_stream), raw(reaction_stream)))


def misdc_get_stats(integ):
    """Statistics of the last step; "converged" is False where the library
    returned MISDC_ENOTCONV (the counts are filled either way)."""
    s = misdc_stats()
    code = lib().misdc_get_stats(integ, C.byref(s))
    if code not in (MISDC_OK, MISDC_ENOTCONV):
        check(code)
    d = s.as_dict()
    d["converged"] = code == MISDC_OK
    return d


NEWTON_HIST_BINS = 64


def misdc_get_newton_histogram(integ, sweep):
    """Outcomes of the last step's Newton solves in one sweep: a list of 64
    counts, [0] not converged, [v] converged after v linear solves, [63]
    after 63 or more."""
    counts = (C.c_int64 * NEWTON_HIST_BINS)()
    check(lib().misdc_get_newton_histogram(integ, int(sweep), counts))
    return list(counts)


def misdc_reset_profile(integ):
    check(lib().misdc_reset_profile(integ))


def misdc_autotune(integ, state, dt, dt_per_flame=None, reps=3, stream=None):
    t = misdc_tune()
    check(lib().misdc_autotune(integ, _ptr(state), float(dt), _ptr(dt_per_flame), int(reps),
                               C.byref(t), _stream(stream)))
    return t.as_dict()


def misdc_get_tune(integ):
    t = misdc_tune()
    check(lib().misdc_get_tune(integ, C.byref(t)))
    return t.as_dict()


def misdc_set_tune(integ, cg_variant, cg_blocks, cyclic, serialize, cu_split=0, stagger=0,
                   fused=0):
    t = misdc_tune(int(cg_variant), int(cg_blocks), int(cyclic), int(serialize), int(cu_split),
                   int(stagger), 0.0, int(fused))
    check(lib().misdc_set_tune(integ, C.byref(t)))


def misdc_mlp_create(n_in, n_hidden, n_out, precision="bf16"):
    h = C.c_void_p()
    check(lib().misdc_mlp_create(int(n_in), int(n_hidden), int(n_out),
                                 MLP_PRECISION[precision], C.byref(h)))
    return h.value


def misdc_mlp_destroy(h):
    check(lib().misdc_mlp_destroy(h))


def misdc_mlp_param_count(h):
    n = C.c_int64()
    check(lib().misdc_mlp_param_count(h, C.byref(n)))
    return n.value


def misdc_mlp_set_params(h, flat):
    a = np.ascontiguousarray(flat, dtype=np.float32)
    check(lib().misdc_mlp_set_params(h, _ptr(a)))


def misdc_mlp_get_params(h):
    a = np.empty(misdc_mlp_param_count(h), dtype=np.float32)
    check(lib().misdc_mlp_get_params(h, _ptr(a)))
    return a


def misdc_mlp_set_normalization(h, in_mu, in_sd, out_sd):
    a, b, c = (np.ascontiguousarray(v, dtype=np.float32) for v in (in_mu, in_sd, out_sd))
    check(lib().misdc_mlp_set_normalization(h, _ptr(a), _ptr(b), _ptr(c)))


def misdc_mlp_forward(h, batch, x, y, stream=None):
    check(lib().misdc_mlp_forward(h, int(batch), _ptr(x), _ptr(y), _stream(stream)))


def misdc_mlp_gradients(h, batch, x, t, grad, loss=None, stream=None):
    check(lib().misdc_mlp_gradients(h, int(batch), _ptr(x), _ptr(t), _ptr(grad), _ptr(loss),
                                    _stream(stream)))


def misdc_mlp_adam_step(h, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check(lib().misdc_mlp_adam_step(h, _ptr(grad), lr, beta1, beta2, eps, _stream(stream)))


def misdc_mlp_train(h, n, x, t, batch, epochs, lr, loss=None, stream=None):
    check(lib().misdc_mlp_train(h, int(n), _ptr(x), _ptr(t), int(batch), int(epochs), float(lr),
                                _ptr(loss), _stream(stream)))


def misdc_mlp_features(mech, h, n, bY, hh, c, x, stream=None):
    check(lib().misdc_mlp_features(mech, h, int(n), _ptr(bY), _ptr(hh), _ptr(c), _ptr(x),
                                   _stream(stream)))


def misdc_mlp_targets(mech, h, n, bY, hh, Y, t, stream=None):
    check(lib().misdc_mlp_targets(mech, h, int(n), _ptr(bY), _ptr(hh), _ptr(Y), _ptr(t),
                                  _stream(stream)))


def misdc_mlp_prepare_training(mech, h, n, bY, hh, c, Y, seed, x, t, stream=None):
    check(lib().misdc_mlp_prepare_training(mech, h, int(n), _ptr(bY), _ptr(hh), _ptr(c), _ptr(Y),
                                           int(seed) & (2**64 - 1), _ptr(x), _ptr(t),
                                           _stream(stream)))


def misdc_reaction_guess_mlp(mech, h, n, bY, hh, c, Y, choice=None, stream=None):
    check(lib().misdc_reaction_guess_mlp(mech, h, int(n), _ptr(bY), _ptr(hh), _ptr(c), _ptr(Y),
                                         _ptr(choice), _stream(stream)))


def misdc_integ_set_guess(integ, mlp, sweeps=0):
    check(lib().misdc_integ_set_guess(integ, mlp, int(sweeps)))


def misdc_integ_record(integ, buf, max_tasks):
    check(lib().misdc_integ_record(integ, _ptr(buf), int(max_tasks)))


def misdc_integ_recorded(integ):
    n = C.c_int64()
    check(lib().misdc_integ_recorded(integ, C.byref(n)))
    return n.value


def make_opts(n_nodes=5, sweeps=6, nu=1, scheme="cisdcq", qe="cumulative", serialize=False,
              cg_rtol=1e-13, cg_maxit=500, newton=None, profile=False, use_graph=False,
              nu_tol=0.0, pipeline=False, imexq_tol=0.0, imexq_maxit=0, imexq_krylov_rtol=0.0,
              imexq_krylov_maxit=0):
    o = misdc_opts_default()
    o.n_nodes = n_nodes
    o.n_sweeps = sweeps
    o.nu = nu
    o.scheme = SCHEME[scheme]
    o.qe_mode = QE[qe]
    o.serialize = int(bool(serialize))
    o.cg_rtol = cg_rtol
    o.cg_maxit = cg_maxit
    o.profile = int(bool(profile))
    o.use_graph = int(bool(use_graph))
    o.nu_tol = float(nu_tol)
    o.pipeline = int(bool(pipeline))
    o.imexq_tol = float(imexq_tol)
    o.imexq_maxit = int(imexq_maxit)
    o.imexq_krylov_rtol = float(imexq_krylov_rtol)
    o.imexq_krylov_maxit = int(imexq_krylov_maxit)
    if newton is not None:
        o.newton = newton
    return o
