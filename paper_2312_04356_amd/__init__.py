"""Python binding of libneujeans.so: the fused CinS-conv + CoeffToSlot hot path on MI355X.

Argument marshalling only: every step runs in the library's HIP kernels (or its
host plan builder).  Device buffers are torch tensors of dtype int64 holding
uint64 residues; streams are torch streams.  There is no fallback: importing
this package fails if the library has not been built.
"""
import ctypes
import os

import numpy as np
# torch first: the library's HIP runtime then binds to the HSA runtime torch loaded,
# and device buffers (torch tensors) and library kernels share one runtime state
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libneujeans.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libneujeans.so is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                      "or `python paper_2312_04356_amd/build_lib.py`")

_lib = ctypes.CDLL(LIB_PATH)

u64, i32, u32, dbl, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p


class NjParams(ctypes.Structure):
    _fields_ = [("log_n", i32), ("n_q", i32), ("alpha", i32), ("q", vp), ("p", vp), ("scale", dbl)]


class NjCt(ctypes.Structure):
    _fields_ = [("data", vp), ("level", i32), ("is_ntt", i32), ("scale", dbl)]


class NjJob(ctypes.Structure):
    _fields_ = [("conv", vp), ("inp", NjCt), ("re", NjCt), ("im", NjCt)]


class NjTap(ctypes.Structure):
    _fields_ = [("out_ch", i32), ("in_ch", i32), ("dy", i32), ("dx", i32), ("w", dbl)]


class NjConvDesc(ctypes.Structure):
    _fields_ = [("w0", i32), ("c_in", i32), ("c_out", i32), ("f", i32), ("stride", i32), ("depthwise", i32),
                ("fuse", i32)]


_SIGS = {
    "nj_last_error": (ctypes.c_char_p, []),
    "nj_gen_primes": (i32, [i32, i32, i32, vp, i32, vp]),
    "nj_ctx_create": (i32, [ctypes.POINTER(NjParams), ctypes.POINTER(vp)]),
    "nj_ctx_destroy": (None, [vp]),
    "nj_set_secret": (i32, [vp, vp]),
    "nj_gen_switch_key": (i32, [vp, u32, vp, vp]),
    "nj_galois_elt": (u32, [vp, i32]),
    "nj_ntt_limbs": (i32, [vp, vp, vp, i32, i32, vp]),
    "nj_to_eval": (i32, [vp, vp, i32, i32, vp]),
    "nj_to_coeff": (i32, [vp, vp, i32, i32, vp]),
    "nj_encrypt_sk": (i32, [vp, vp, i32, vp, vp, dbl, ctypes.POINTER(NjCt), vp]),
    "nj_key_words": (ctypes.c_size_t, [vp]),
    "nj_key_export": (i32, [vp, u32, vp, ctypes.c_size_t]),
    "nj_key_import": (i32, [vp, u32, vp, ctypes.c_size_t]),
    "nj_key_list": (i32, [vp, vp, i32, ctypes.POINTER(i32)]),
    "nj_gen_public_key": (i32, [vp, vp, vp]),
    "nj_encrypt_pk": (i32, [vp, vp, i32, vp, vp, vp, dbl, ctypes.POINTER(NjCt), vp]),
    "nj_decrypt": (i32, [vp, ctypes.POINTER(NjCt), vp, vp]),
    "nj_encode_slots": (i32, [i32, vp, dbl, vp]),
    "nj_encode_cins": (i32, [i32, vp, i32, dbl, vp]),
    "nj_decode_slots": (i32, [i32, vp, dbl, vp]),
    "nj_upload_plain": (i32, [vp, vp, i32, vp, vp]),
    "nj_rotate": (i32, [vp, ctypes.POINTER(NjCt), i32, ctypes.POINTER(NjCt), vp]),
    "nj_apply_galois": (i32, [vp, ctypes.POINTER(NjCt), u32, ctypes.POINTER(NjCt), vp]),
    "nj_apply_galois_noalloc": (i32, [vp, ctypes.POINTER(NjCt), u32, ctypes.POINTER(NjCt), vp]),
    "nj_keyswitch": (i32, [vp, vp, i32, u32, vp, vp, vp]),
    "nj_pmult": (i32, [vp, ctypes.POINTER(NjCt), vp, ctypes.POINTER(NjCt), vp]),
    "nj_add": (i32, [vp, ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), vp]),
    "nj_sub": (i32, [vp, ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), vp]),
    "nj_rescale": (i32, [vp, ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), vp]),
    "nj_modraise": (i32, [vp, ctypes.POINTER(NjCt), i32, ctypes.POINTER(NjCt), vp]),
    "nj_plan_count": (i32, [vp]),
    "nj_plan_galois": (i32, [vp, vp, i32]),
    "nj_plan_offsets": (i32, [vp, i32, vp, i32]),
    "nj_plan_set_diagonal": (i32, [vp, vp, i32, i32, vp]),
    "nj_plan_destroy": (None, [vp]),
    "nj_conv_plan_create": (i32, [vp, i32, i32, vp, i32, ctypes.POINTER(vp)]),
    "nj_cts_plan_create": (i32, [vp, i32, ctypes.POINTER(vp)]),
    "nj_conv_plan_create_taps": (i32, [vp, i32, i32, i32, vp, i32, i32, i32, i32, ctypes.POINTER(vp)]),
    "nj_conv_taps": (i32, [i32, i32, i32, i32, i32, vp, vp, i32, ctypes.POINTER(i32)]),
    "nj_downsample_plan_create": (i32, [vp, i32, i32, i32, i32, i32, i32, ctypes.POINTER(vp)]),
    "nj_fc_plan_create": (i32, [vp, i32, i32, vp, i32, i32, ctypes.POINTER(vp)]),
    "nj_conv_plan_create_layer": (i32, [vp, ctypes.POINTER(NjConvDesc), vp, i32, i32, ctypes.POINTER(vp)]),
    "nj_plan_layout": (i32, [vp, vp, vp, vp, vp, vp]),
    "nj_conv2d_block": (i32, [vp, vp, ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), vp]),
    "nj_drop_level": (i32, [vp, ctypes.POINTER(NjCt), i32, ctypes.POINTER(NjCt), vp]),
    "nj_batch_run": (i32, [vp, vp, vp, i32, i32, vp]),
    "nj_batch_workers": (i32, [vp, i32]),
    "nj_batch_create_mode": (i32, [vp, vp, vp, i32, i32, ctypes.POINTER(vp)]),
    "nj_batch_create": (i32, [vp, vp, vp, i32, ctypes.POINTER(vp)]),
    "nj_batch_launch": (i32, [vp, vp]),
    "nj_batch_destroy": (None, [vp]),
    "nj_timing_keys": (i32, [vp, i32]),
    "nj_plan_set_lazy": (i32, [vp, i32]),
    "nj_plan_set_hoist": (i32, [vp, i32, i32]),
    "nj_cts_plan_create_split": (i32, [vp, i32, vp, ctypes.POINTER(vp)]),
    "nj_cts_plan_features": (i32, [vp, i32, vp, i32, vp]),
    "nj_hmult": (i32, [vp, ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), vp]),
    "nj_mul_const": (i32, [vp, ctypes.POINTER(NjCt), dbl, i32, dbl, ctypes.POINTER(NjCt), vp]),
    "nj_add_const": (i32, [vp, ctypes.POINTER(NjCt), dbl, vp]),
    "nj_cheb_interpolate": (i32, [i32, dbl, i32, vp]),
    "nj_eval_mod": (i32, [vp, ctypes.POINTER(NjCt), i32, i32, vp, i32, ctypes.POINTER(NjCt), vp]),
    "nj_eval_order": (i32, [vp, i32]),
    "nj_combine": (i32, [vp, ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), vp]),
    "nj_stoc1_plan_create": (i32, [vp, i32, i32, i32, ctypes.POINTER(vp)]),
    "nj_stoc1": (i32, [vp, vp, ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), vp]),
    "nj_layer_masks": (i32, [i32, i32, i32, i32, vp, vp]),
    "nj_slot_activation": (i32, [vp, i32, i32, vp, i32, vp, vp, i32, vp, ctypes.POINTER(NjCt), ctypes.POINTER(NjCt),
                                 ctypes.POINTER(NjCt), vp]),
    "nj_slot_activation_decompose": (i32, [vp, i32, i32, vp, i32, vp, vp, i32, vp, vp, vp, ctypes.POINTER(NjCt),
                                           ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), vp]),
    "nj_conv_act_layer": (i32, [vp, vp, vp, i32, i32, vp, i32, vp, vp, i32, vp, ctypes.POINTER(NjCt),
                                ctypes.POINTER(NjCt), vp]),
    "nj_bootstrap": (i32, [vp, vp, i32, i32, vp, i32, vp, ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), vp]),
    "nj_plan_create_random": (i32, [vp, i32, i32, vp, i32, i32, i32, i32, u64, ctypes.POINTER(vp)]),
    "nj_time_plan": (i32, [vp, vp, i32, i32, i32, ctypes.POINTER(ctypes.c_float)]),
    "nj_plan_features": (i32, [vp, i32, i32, vp]),
    "nj_tune_split": (i32, [vp, vp, i32, i32, vp, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), vp,
                            ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "nj_mlp_create": (i32, [u64, ctypes.POINTER(vp)]),
    "nj_mlp_destroy": (None, [vp]),
    "nj_mlp_set_params": (i32, [vp, vp]),
    "nj_mlp_get_params": (i32, [vp, vp]),
    "nj_mlp_get_norm": (i32, [vp, vp]),
    "nj_mlp_set_norm": (i32, [vp, vp]),
    "nj_mlp_grad": (i32, [vp, vp, vp, i32, vp, ctypes.POINTER(ctypes.c_float)]),
    "nj_mlp_train": (i32, [vp, vp, vp, i32, i32, i32, ctypes.c_float, u64, ctypes.POINTER(ctypes.c_float)]),
    "nj_mlp_predict": (i32, [vp, vp, i32, vp]),
    "nj_plan_apply": (i32, [vp, vp, i32, ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), i32, vp]),
    "nj_conv2d_cins": (i32, [vp, vp, ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), vp]),
    "nj_coeff_to_slot": (i32, [vp, vp, ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), ctypes.POINTER(NjCt), vp]),
    "nj_apply_galois_batch": (i32, [vp, ctypes.POINTER(NjCt), i32, u32, ctypes.POINTER(NjCt), vp]),
    "nj_conv2d_cins_batch": (i32, [vp, vp, ctypes.POINTER(NjCt), i32, ctypes.POINTER(NjCt), vp]),
    "nj_coeff_to_slot_batch": (i32, [vp, vp, ctypes.POINTER(NjCt), i32, ctypes.POINTER(NjCt),
                                     ctypes.POINTER(NjCt), vp]),
    "nj_prof_enable": (i32, [vp, i32]),
    "nj_prof_read": (i32, [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl), ctypes.POINTER(dbl), i32]),
}

# live-profiled kernel families (nj_prof_read kinds) and the kernel names rocprofv3 reports for them
PROF_KERNELS = {0: "k_ntt_tile<false>", 1: "k_ntt_tile<true>", 2: "k_ntt_col<false>", 3: "k_ntt_col<true>",
                4: "k_bconv", 5: "k_key_ip", 6: "k_pmac", 7: "other", 8: "k_ntt_tile_md"}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = sorted(_SIGS)


class NjError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib.nj_last_error().decode(errors="replace")
        super().__init__("%s failed (status %d): %s" % (where, code, msg))
        self.code = code


def _check(code, where):
    if code != 0:
        raise NjError(code, where)


def _np_ptr(a):
    return a.ctypes.data_as(vp)


def _dev_ptr(t):
    return vp(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return vp(s.cuda_stream)


# ------------------------------------------------------------------ host-only

def nj_gen_primes(log_n, bits, count, exclude=()):
    ex = np.ascontiguousarray(np.array(list(exclude) or [0], dtype=np.uint64))
    out = np.zeros(count, dtype=np.uint64)
    _check(_lib.nj_gen_primes(log_n, bits, count, _np_ptr(ex), len(exclude), _np_ptr(out)), "nj_gen_primes")
    return [int(x) for x in out]


def nj_encode_slots(log_n, z, scale):
    zz = np.ascontiguousarray(np.stack([np.real(z), np.imag(z)], axis=-1), dtype=np.float64)
    out = np.zeros(1 << log_n, dtype=np.int64)
    _check(_lib.nj_encode_slots(log_n, _np_ptr(zz), float(scale), _np_ptr(out)), "nj_encode_slots")
    return out


def nj_encode_cins(log_n, chans, scale):
    ch = np.ascontiguousarray(chans, dtype=np.float64)
    out = np.zeros(1 << log_n, dtype=np.int64)
    _check(_lib.nj_encode_cins(log_n, _np_ptr(ch), ch.shape[-1], float(scale), _np_ptr(out)), "nj_encode_cins")
    return out


def nj_decode_slots(log_n, coeffs, scale):
    cf = np.ascontiguousarray(coeffs, dtype=np.float64)
    z = np.zeros(((1 << log_n) // 2, 2), dtype=np.float64)
    _check(_lib.nj_decode_slots(log_n, _np_ptr(cf), float(scale), _np_ptr(z)), "nj_decode_slots")
    return z[:, 0] + 1j * z[:, 1]


def chain_primes(log_n, n_q, alpha, q0_bits, q_bits, p_bits):
    """q_0 (q0_bits), q_1.. (q_bits), p_0.. (p_bits): each the next unused prime of the chain rule."""
    q0 = nj_gen_primes(log_n, q0_bits, 1)
    qs = nj_gen_primes(log_n, q_bits, n_q - 1, q0)
    ps = nj_gen_primes(log_n, p_bits, alpha, q0 + qs)
    return q0 + qs, ps


# ------------------------------------------------------------------- objects

class Ct:
    """A device ciphertext [2][level+1][N] (torch int64 tensor of uint64 residues)."""

    def __init__(self, data, level, is_ntt=1, scale=1.0):
        self.data, self.level, self.is_ntt, self.scale = data, level, is_ntt, scale

    def c(self):
        return NjCt(self.data.data_ptr(), self.level, self.is_ntt, self.scale)

    def sync_from(self, s):
        self.level, self.is_ntt, self.scale = s.level, s.is_ntt, s.scale
        return self


class Plan:
    def __init__(self, ptr):
        self.ptr = ptr

    def count(self):
        return _lib.nj_plan_count(self.ptr)

    def galois(self):
        buf = np.zeros(4096, dtype=np.uint32)
        n = _lib.nj_plan_galois(self.ptr, _np_ptr(buf), 4096)
        return [int(x) for x in buf[:n]]

    def layout(self):
        """(level, W, C, l, bi, bo) of a conv plan"""
        v = [i32() for _ in range(5)]
        lvl = _lib.nj_plan_layout(self.ptr, *[ctypes.byref(x) for x in v])
        return (lvl,) + tuple(x.value for x in v)

    def set_lazy(self, on=True):
        _check(_lib.nj_plan_set_lazy(self.ptr, int(bool(on))), "nj_plan_set_lazy")
        return self

    def set_hoist(self, on=True, t=-1):
        """hoisted baby steps for transform t (-1: all); on may be a list, one per transform"""
        if isinstance(on, (list, tuple)):
            for i, v in enumerate(on):
                _check(_lib.nj_plan_set_hoist(self.ptr, i, int(bool(v))), "nj_plan_set_hoist")
        else:
            _check(_lib.nj_plan_set_hoist(self.ptr, int(t), int(bool(on))), "nj_plan_set_hoist")
        return self

    def features(self, level, t=0):
        f = np.zeros(7, dtype=np.float32)
        _check(_lib.nj_plan_features(self.ptr, int(t), int(level), _np_ptr(f)), "nj_plan_features")
        return f

    def offsets(self, t):
        buf = np.zeros(1 << 16, dtype=np.int32)
        n = _lib.nj_plan_offsets(self.ptr, t, _np_ptr(buf), 1 << 16)
        return [int(x) for x in buf[:n]]

    def __del__(self):
        if getattr(self, "ptr", None):
            _lib.nj_plan_destroy(self.ptr)
            self.ptr = None


def nj_conv_taps(K, stride=1, depthwise=False):
    """the library's taps (out, in, dy, dx, w) of a conv layer with weights K
    [c_out][c_in][f][f] (depthwise: [c][f][f])"""
    K = np.ascontiguousarray(K, dtype=np.float64)
    if depthwise:
        c_out = c_in = K.shape[0]
    else:
        c_out, c_in = K.shape[0], K.shape[1]
    f = K.shape[-1]
    n = i32()
    _check(_lib.nj_conv_taps(c_in, c_out, f, int(stride), int(bool(depthwise)), _np_ptr(K), None, 0, ctypes.byref(n)),
           "nj_conv_taps")
    arr = (NjTap * n.value)()
    _check(_lib.nj_conv_taps(c_in, c_out, f, int(stride), int(bool(depthwise)), _np_ptr(K), ctypes.cast(arr, vp),
                             n.value, ctypes.byref(n)), "nj_conv_taps")
    return [(t.out_ch, t.in_ch, t.dy, t.dx, t.w) for t in arr]


def nj_layer_masks(log_n, W, C, w0):
    """(mask_re, mask_im): Algorithm 1's zero-padding slot masks, N/2 doubles each"""
    n2 = 1 << (log_n - 1)
    mre, mim = np.zeros(n2), np.zeros(n2)
    _check(_lib.nj_layer_masks(int(log_n), int(W), int(C), int(w0), _np_ptr(mre), _np_ptr(mim)), "nj_layer_masks")
    return mre, mim


def _coeffs(coeffs):
    return None if coeffs is None else np.ascontiguousarray(coeffs, dtype=np.float64)


def nj_cheb_interpolate(degree, K, r):
    out = np.zeros(degree + 1, dtype=np.float64)
    _check(_lib.nj_cheb_interpolate(int(degree), float(K), int(r), _np_ptr(out)), "nj_cheb_interpolate")
    return out


MLP_FEATURES, MLP_HIDDEN = 7, 64
MLP_PARAMS = 7 * 64 + 64 + 64 * 64 + 64 + 64 + 1
MLP_NORM = 2 * 7 + 2


class Mlp:
    """nj_mlp: the 7 -> 64 -> 64 -> 1 FP32 latency model (trained and evaluated on the GPU)."""

    def __init__(self, seed=0):
        h = vp()
        _check(_lib.nj_mlp_create(u64(seed), ctypes.byref(h)), "nj_mlp_create")
        self.ptr = h

    def params(self):
        out = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(_lib.nj_mlp_get_params(self.ptr, _np_ptr(out)), "nj_mlp_get_params")
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.shape == (MLP_PARAMS,)
        _check(_lib.nj_mlp_set_params(self.ptr, _np_ptr(p)), "nj_mlp_set_params")

    def norm(self):
        out = np.zeros(MLP_NORM, dtype=np.float32)
        _check(_lib.nj_mlp_get_norm(self.ptr, _np_ptr(out)), "nj_mlp_get_norm")
        return out

    def set_norm(self, v):
        v = np.ascontiguousarray(v, dtype=np.float32)
        assert v.shape == (MLP_NORM,)
        _check(_lib.nj_mlp_set_norm(self.ptr, _np_ptr(v)), "nj_mlp_set_norm")

    def to_dict(self):
        """the trained model as plain lists (JSON-serialisable)"""
        return {"params": [float(x) for x in self.params()], "norm": [float(x) for x in self.norm()]}

    @classmethod
    def from_dict(cls, d):
        m = cls(0)
        m.set_params(np.array(d["params"], dtype=np.float32))
        m.set_norm(np.array(d["norm"], dtype=np.float32))
        return m

    def grad(self, X, y):
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        loss = ctypes.c_float()
        _check(_lib.nj_mlp_grad(self.ptr, _np_ptr(X), _np_ptr(y), len(y), _np_ptr(g), ctypes.byref(loss)),
               "nj_mlp_grad")
        return g, loss.value

    def train(self, X, y, epochs=200, batch=256, lr=1e-3, seed=0):
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        loss = ctypes.c_float()
        _check(_lib.nj_mlp_train(self.ptr, _np_ptr(X), _np_ptr(y), len(y), int(epochs), int(batch), float(lr),
                                 u64(seed), ctypes.byref(loss)), "nj_mlp_train")
        return loss.value

    def predict(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        out = np.zeros(X.shape[0], dtype=np.float32)
        _check(_lib.nj_mlp_predict(self.ptr, _np_ptr(X), X.shape[0], _np_ptr(out)), "nj_mlp_predict")
        return out

    def __del__(self):
        if getattr(self, "ptr", None):
            _lib.nj_mlp_destroy(self.ptr)
            self.ptr = None


class Batch:
    """nj_batch: a captured HIP graph of a batched job list (holds its plans and buffers)."""

    def __init__(self, ptr, keep):
        self.ptr, self.keep = ptr, keep

    def launch(self, stream=None):
        _check(_lib.nj_batch_launch(self.ptr, _stream(stream)), "nj_batch_launch")

    def __del__(self):
        if getattr(self, "ptr", None):
            _lib.nj_batch_destroy(self.ptr)
            self.ptr = None


class Ctx:
    """nj_ctx: ring, primes, tables, secret, switching keys."""

    def __init__(self, log_n, q, p, scale, device=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", 0) if device is None else device
        torch.cuda.set_device(self.device)
        self.N = 1 << log_n
        self.log_n = log_n
        self.q, self.p = [int(x) for x in q], [int(x) for x in p]
        self.L = len(self.q) - 1
        self.alpha = len(self.p)
        self.scale = scale
        self._qa = np.array(self.q, dtype=np.uint64)
        self._pa = np.array(self.p, dtype=np.uint64)
        prm = NjParams(log_n, len(self.q), len(self.p), self._qa.ctypes.data, self._pa.ctypes.data, scale)
        h = vp()
        _check(_lib.nj_ctx_create(ctypes.byref(prm), ctypes.byref(h)), "nj_ctx_create")
        self.ptr = h

    def __del__(self):
        if getattr(self, "ptr", None):
            _lib.nj_ctx_destroy(self.ptr)
            self.ptr = None

    @property
    def dnum(self):
        return -(-(self.L + 1) // self.alpha)

    def empty_ct(self, level):
        t = self.torch.empty((2, level + 1, self.N), dtype=self.torch.int64, device=self.device)
        return Ct(t, level)

    def to_device(self, arr):
        a = np.ascontiguousarray(arr).view(np.int64)
        return self.torch.from_numpy(a.copy()).to(self.device)

    @staticmethod
    def to_host(t):
        return t.detach().cpu().numpy().view(np.uint64)

    # -- keys
    def nj_set_secret(self, s):
        s8 = np.ascontiguousarray(s, dtype=np.int8)
        _check(_lib.nj_set_secret(self.ptr, _np_ptr(s8)), "nj_set_secret")
        self.secret = s8.copy()

    def nj_gen_switch_key(self, g, a, e):
        a = np.ascontiguousarray(a, dtype=np.uint64)
        e = np.ascontiguousarray(e, dtype=np.int64)
        assert a.shape == (self.dnum, self.L + 1 + self.alpha, self.N) and e.shape == (self.dnum, self.N)
        _check(_lib.nj_gen_switch_key(self.ptr, int(g), _np_ptr(a), _np_ptr(e)), "nj_gen_switch_key")

    def nj_galois_elt(self, r):
        return int(_lib.nj_galois_elt(self.ptr, int(r)))

    # -- transforms
    def nj_ntt_limbs(self, data, prime_idx, inverse, stream=None):
        pi = np.ascontiguousarray(prime_idx, dtype=np.int32)
        _check(_lib.nj_ntt_limbs(self.ptr, _dev_ptr(data), _np_ptr(pi), len(pi), int(inverse), _stream(stream)),
               "nj_ntt_limbs")

    def nj_to_eval(self, data, level, n_polys, stream=None):
        _check(_lib.nj_to_eval(self.ptr, _dev_ptr(data), level, n_polys, _stream(stream)), "nj_to_eval")

    def nj_to_coeff(self, data, level, n_polys, stream=None):
        _check(_lib.nj_to_coeff(self.ptr, _dev_ptr(data), level, n_polys, _stream(stream)), "nj_to_coeff")

    # -- encryption / encoding
    def nj_encrypt_sk(self, m_dev, level, a, e, scale, out, stream=None):
        a = np.ascontiguousarray(a, dtype=np.uint64)
        e = np.ascontiguousarray(e, dtype=np.int64)
        assert a.shape == (level + 1, self.N) and e.shape == (self.N,)
        c = out.c()
        _check(_lib.nj_encrypt_sk(self.ptr, _dev_ptr(m_dev), level, _np_ptr(a), _np_ptr(e), float(scale),
                                  ctypes.byref(c), _stream(stream)), "nj_encrypt_sk")
        return out.sync_from(c)

    # -- switching keys in and out (saving and restoring a key set)
    def nj_key_words(self):
        return int(_lib.nj_key_words(self.ptr))

    def nj_key_list(self):
        n = i32()
        _check(_lib.nj_key_list(self.ptr, None, 0, ctypes.byref(n)), "nj_key_list")
        out = np.zeros(max(1, n.value), dtype=np.uint32)
        _check(_lib.nj_key_list(self.ptr, _np_ptr(out), len(out), ctypes.byref(n)), "nj_key_list")
        return [int(g) for g in out[:n.value]]

    def nj_key_export(self, g):
        out = np.empty(self.nj_key_words(), dtype=np.uint64)
        _check(_lib.nj_key_export(self.ptr, int(g), _np_ptr(out), out.size), "nj_key_export")
        return out

    def nj_key_import(self, g, words):
        w = np.ascontiguousarray(words, dtype=np.uint64)
        _check(_lib.nj_key_import(self.ptr, int(g), _np_ptr(w), w.size), "nj_key_import")

    def key_fingerprint(self):
        """what a saved key is tied to: ring degree, primes, digit size and the secret's
        hash (keys only decrypt under the secret that made them)"""
        import hashlib
        sec = hashlib.sha256(np.ascontiguousarray(self.secret, dtype=np.int8).tobytes()).hexdigest() \
            if getattr(self, "secret", None) is not None else ""
        return {"N": self.N, "q": [int(x) for x in self.q], "p": [int(x) for x in self.p],
                "alpha": int(self.alpha), "secret_sha256": sec}

    def save_keys(self, path, gs=None):
        """every switching key (or those of gs) to an .npz file with the fingerprint"""
        import json
        gs = self.nj_key_list() if gs is None else list(gs)
        arrays = {"key_%d" % g: self.nj_key_export(g) for g in gs}
        np.savez(path, fingerprint=np.frombuffer(json.dumps(self.key_fingerprint()).encode(), dtype=np.uint8),
                 **arrays)
        return gs

    def load_keys(self, path):
        """keys saved by save_keys into this context; ValueError if the file was written
        for other parameters or another secret"""
        import json
        with np.load(path, allow_pickle=False) as f:
            fp = json.loads(bytes(f["fingerprint"]).decode())
            if fp != self.key_fingerprint():
                raise ValueError("saved keys belong to other parameters or another secret")
            gs = sorted(int(k[4:]) for k in f.files if k.startswith("key_"))
            for g in gs:
                self.nj_key_import(g, f["key_%d" % g])
        return gs

    def nj_gen_public_key(self, a, e):
        a = np.ascontiguousarray(a, dtype=np.uint64)
        e = np.ascontiguousarray(e, dtype=np.int64)
        assert a.shape == (self.L + 1, self.N) and e.shape == (self.N,)
        _check(_lib.nj_gen_public_key(self.ptr, _np_ptr(a), _np_ptr(e)), "nj_gen_public_key")

    def nj_encrypt_pk(self, m_dev, level, v, e0, e1, scale, out, stream=None):
        v, e0, e1 = (np.ascontiguousarray(x, dtype=np.int64) for x in (v, e0, e1))
        assert v.shape == e0.shape == e1.shape == (self.N,)
        c = out.c()
        _check(_lib.nj_encrypt_pk(self.ptr, _dev_ptr(m_dev), level, _np_ptr(v), _np_ptr(e0), _np_ptr(e1),
                                  float(scale), ctypes.byref(c), _stream(stream)), "nj_encrypt_pk")
        return out.sync_from(c)

    def nj_decrypt(self, ct, out_dev, stream=None):
        c = ct.c()
        _check(_lib.nj_decrypt(self.ptr, ctypes.byref(c), _dev_ptr(out_dev), _stream(stream)), "nj_decrypt")

    def nj_encode_slots(self, z, scale):
        return nj_encode_slots(self.log_n, z, scale)

    def nj_encode_cins(self, chans, scale):
        return nj_encode_cins(self.log_n, chans, scale)

    def nj_decode_slots(self, coeffs, scale):
        return nj_decode_slots(self.log_n, coeffs, scale)

    def nj_upload_plain(self, coeffs, level, dst, stream=None):
        cf = np.ascontiguousarray(coeffs, dtype=np.int64)
        _check(_lib.nj_upload_plain(self.ptr, _np_ptr(cf), level, _dev_ptr(dst), _stream(stream)), "nj_upload_plain")

    # -- homomorphic ops
    def nj_rotate(self, ct, r, out, stream=None):
        ci, co = ct.c(), out.c()
        _check(_lib.nj_rotate(self.ptr, ctypes.byref(ci), int(r), ctypes.byref(co), _stream(stream)), "nj_rotate")
        return out.sync_from(co)

    def nj_apply_galois(self, ct, g, out, stream=None):
        ci, co = ct.c(), out.c()
        _check(_lib.nj_apply_galois(self.ptr, ctypes.byref(ci), int(g), ctypes.byref(co), _stream(stream)),
               "nj_apply_galois")
        return out.sync_from(co)

    def nj_apply_galois_noalloc(self, ct, g, out, stream=None):
        ci, co = ct.c(), out.c()
        _check(_lib.nj_apply_galois_noalloc(self.ptr, ctypes.byref(ci), int(g), ctypes.byref(co), _stream(stream)),
               "nj_apply_galois_noalloc")
        return out.sync_from(co)

    def nj_keyswitch(self, d, level, g, out0, out1, stream=None):
        _check(_lib.nj_keyswitch(self.ptr, _dev_ptr(d), level, int(g), _dev_ptr(out0), _dev_ptr(out1),
                                 _stream(stream)), "nj_keyswitch")

    def nj_pmult(self, ct, pt_dev, out, stream=None):
        ci, co = ct.c(), out.c()
        _check(_lib.nj_pmult(self.ptr, ctypes.byref(ci), _dev_ptr(pt_dev), ctypes.byref(co), _stream(stream)),
               "nj_pmult")
        return out.sync_from(co)

    def nj_add(self, a, b, out, stream=None):
        ca, cb, co = a.c(), b.c(), out.c()
        _check(_lib.nj_add(self.ptr, ctypes.byref(ca), ctypes.byref(cb), ctypes.byref(co), _stream(stream)), "nj_add")
        return out.sync_from(co)

    def nj_sub(self, a, b, out, stream=None):
        ca, cb, co = a.c(), b.c(), out.c()
        _check(_lib.nj_sub(self.ptr, ctypes.byref(ca), ctypes.byref(cb), ctypes.byref(co), _stream(stream)), "nj_sub")
        return out.sync_from(co)

    def nj_rescale(self, ct, out, stream=None):
        ci, co = ct.c(), out.c()
        _check(_lib.nj_rescale(self.ptr, ctypes.byref(ci), ctypes.byref(co), _stream(stream)), "nj_rescale")
        return out.sync_from(co)

    def nj_modraise(self, ct, level, out, stream=None):
        ci, co = ct.c(), out.c()
        _check(_lib.nj_modraise(self.ptr, ctypes.byref(ci), level, ctypes.byref(co), _stream(stream)), "nj_modraise")
        return out.sync_from(co)

    # -- batched calls (Ct data tensors of shape [n, 2, level+1, N])
    def empty_batch(self, n, level):
        t = self.torch.empty((n, 2, level + 1, self.N), dtype=self.torch.int64, device=self.device)
        return Ct(t, level)

    def nj_apply_galois_batch(self, ct, n, g, out, stream=None):
        ci, co = ct.c(), out.c()
        _check(_lib.nj_apply_galois_batch(self.ptr, ctypes.byref(ci), int(n), int(g), ctypes.byref(co),
                                          _stream(stream)), "nj_apply_galois_batch")
        return out.sync_from(co)

    def nj_conv2d_cins_batch(self, plan, ct, n, out, stream=None):
        ci, co = ct.c(), out.c()
        _check(_lib.nj_conv2d_cins_batch(self.ptr, plan.ptr, ctypes.byref(ci), int(n), ctypes.byref(co),
                                         _stream(stream)), "nj_conv2d_cins_batch")
        return out.sync_from(co)

    def nj_coeff_to_slot_batch(self, plan, ct, n, re, im, stream=None):
        ci, cr, cm = ct.c(), re.c(), im.c()
        _check(_lib.nj_coeff_to_slot_batch(self.ptr, plan.ptr, ctypes.byref(ci), int(n), ctypes.byref(cr),
                                           ctypes.byref(cm), _stream(stream)), "nj_coeff_to_slot_batch")
        re.sync_from(cr)
        im.sync_from(cm)
        return re, im

    # -- profiling
    def nj_prof_enable(self, on):
        _check(_lib.nj_prof_enable(self.ptr, int(on)), "nj_prof_enable")

    def nj_prof_read(self, kind, reset=True):
        n, ms, by = i32(), dbl(), dbl()
        _check(_lib.nj_prof_read(self.ptr, int(kind), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by),
                                 int(reset)), "nj_prof_read")
        return n.value, ms.value, by.value

    # -- plans
    def nj_conv_plan_create(self, w0, f, weights, n1=0):
        w = np.ascontiguousarray(weights, dtype=np.float64)
        h = vp()
        _check(_lib.nj_conv_plan_create(self.ptr, w0, f, _np_ptr(w), n1, ctypes.byref(h)), "nj_conv_plan_create")
        return Plan(h)

    def nj_conv_plan_create_taps(self, w0, c_in, c_out, taps, fuse=1, n1=0, level=1):
        """taps: iterable of (out_ch, in_ch, dy, dx, w)"""
        taps = list(taps)
        arr = (NjTap * len(taps))(*[NjTap(int(o), int(i), int(dy), int(dx), float(w)) for (o, i, dy, dx, w) in taps])
        h = vp()
        _check(_lib.nj_conv_plan_create_taps(self.ptr, int(w0), int(c_in), int(c_out), ctypes.cast(arr, vp),
                                             len(taps), int(fuse), int(n1), int(level), ctypes.byref(h)),
               "nj_conv_plan_create_taps")
        return Plan(h)

    def nj_conv_plan_create_layer(self, w0, K, stride=1, depthwise=False, fuse=1, n1=0, level=1):
        """plan of a conv layer with weights K [c_out][c_in][f][f] (depthwise: [c][f][f]) on
        w0 x w0 inputs (stride 2: inputs in the phase layout)"""
        K = np.ascontiguousarray(K, dtype=np.float64)
        c_out = K.shape[0]
        c_in = c_out if depthwise else K.shape[1]
        d = NjConvDesc(int(w0), int(c_in), int(c_out), int(K.shape[-1]), int(stride), int(bool(depthwise)), int(fuse))
        h = vp()
        _check(_lib.nj_conv_plan_create_layer(self.ptr, ctypes.byref(d), _np_ptr(K), int(n1), int(level),
                                              ctypes.byref(h)), "nj_conv_plan_create_layer")
        return Plan(h)

    def nj_downsample_plan_create(self, kind, W, C, half, level, n1=0):
        """kind 0 decompose / 1 densify slot permutation for one half (0 Re, 1 Im)"""
        h = vp()
        _check(_lib.nj_downsample_plan_create(self.ptr, int(kind), int(W), int(C), int(half), int(n1), int(level),
                                              ctypes.byref(h)), "nj_downsample_plan_create")
        return Plan(h)

    def nj_fc_plan_create(self, weights, level, n1=0):
        """FC layer [n_out][n_in] fused with the whole StoC"""
        w = np.ascontiguousarray(weights, dtype=np.float64)
        h = vp()
        _check(_lib.nj_fc_plan_create(self.ptr, int(w.shape[1]), int(w.shape[0]), _np_ptr(w), int(n1), int(level),
                                      ctypes.byref(h)), "nj_fc_plan_create")
        return Plan(h)

    def nj_conv2d_block(self, plan, ct, out, stream=None):
        ci, co = ct.c(), out.c()
        _check(_lib.nj_conv2d_block(self.ptr, plan.ptr, ctypes.byref(ci), ctypes.byref(co), _stream(stream)),
               "nj_conv2d_block")
        return out.sync_from(co)

    def nj_drop_level(self, ct, level, out, stream=None):
        ci, co = ct.c(), out.c()
        _check(_lib.nj_drop_level(self.ptr, ctypes.byref(ci), int(level), ctypes.byref(co), _stream(stream)),
               "nj_drop_level")
        return out.sync_from(co)

    def _jobs(self, jobs):
        """jobs: [(conv_plan, in_ct, re_ct, im_ct)] -> ctypes array (kept alive by the caller)"""
        arr = (NjJob * len(jobs))()
        for k, (plan, x, re, im) in enumerate(jobs):
            arr[k] = NjJob(plan.ptr, x.c(), re.c(), im.c())
        return arr

    def _sync_jobs(self, jobs, arr):
        for (plan, x, re, im), j in zip(jobs, arr):
            re.sync_from(j.re)
            im.sync_from(j.im)

    def nj_batch_run(self, cts_plan, jobs, mode, stream=None):
        arr = self._jobs(jobs)
        _check(_lib.nj_batch_run(self.ptr, cts_plan.ptr, ctypes.cast(arr, vp), len(jobs), int(mode), _stream(stream)),
               "nj_batch_run")
        self._sync_jobs(jobs, arr)

    def nj_batch_create(self, cts_plan, jobs, mode=1):
        arr = self._jobs(jobs)
        h = vp()
        _check(_lib.nj_batch_create_mode(self.ptr, cts_plan.ptr, ctypes.cast(arr, vp), len(jobs), int(mode),
                                         ctypes.byref(h)), "nj_batch_create_mode")
        self._sync_jobs(jobs, arr)
        return Batch(h, (cts_plan, jobs))

    def nj_batch_workers(self, n):
        _check(_lib.nj_batch_workers(self.ptr, int(n)), "nj_batch_workers")

    # -- bootstrapping after CoeffToSlot
    def nj_hmult(self, a, b, out, stream=None):
        ca, cb, co = a.c(), b.c(), out.c()
        _check(_lib.nj_hmult(self.ptr, ctypes.byref(ca), ctypes.byref(cb), ctypes.byref(co), _stream(stream)),
               "nj_hmult")
        return out.sync_from(co)

    def nj_mul_const(self, ct, v, level, scale, out, stream=None):
        ci, co = ct.c(), out.c()
        _check(_lib.nj_mul_const(self.ptr, ctypes.byref(ci), float(v), int(level), float(scale), ctypes.byref(co),
                                 _stream(stream)), "nj_mul_const")
        return out.sync_from(co)

    def nj_add_const(self, ct, v, stream=None):
        ci = ct.c()
        _check(_lib.nj_add_const(self.ptr, ctypes.byref(ci), float(v), _stream(stream)), "nj_add_const")
        return ct

    def nj_eval_order(self, order):
        _check(_lib.nj_eval_order(self.ptr, int(order)), "nj_eval_order")

    def nj_eval_mod(self, ct, K, r, coeffs, out, stream=None):
        ci, co = ct.c(), out.c()
        cf = None if coeffs is None else np.ascontiguousarray(coeffs, dtype=np.float64)
        _check(_lib.nj_eval_mod(self.ptr, ctypes.byref(ci), int(K), int(r), None if cf is None else _np_ptr(cf),
                                0 if cf is None else len(cf), ctypes.byref(co), _stream(stream)), "nj_eval_mod")
        return out.sync_from(co)

    def nj_combine(self, re, im, out, stream=None):
        cr, cm, co = re.c(), im.c(), out.c()
        _check(_lib.nj_combine(self.ptr, ctypes.byref(cr), ctypes.byref(cm), ctypes.byref(co), _stream(stream)),
               "nj_combine")
        return out.sync_from(co)

    def nj_stoc1_plan_create(self, ell, groups, level):
        h = vp()
        _check(_lib.nj_stoc1_plan_create(self.ptr, int(ell), int(groups), int(level), ctypes.byref(h)),
               "nj_stoc1_plan_create")
        return Plan(h)

    def nj_stoc1(self, plan, ct, out, stream=None):
        ci, co = ct.c(), out.c()
        _check(_lib.nj_stoc1(self.ptr, plan.ptr, ctypes.byref(ci), ctypes.byref(co), _stream(stream)), "nj_stoc1")
        return out.sync_from(co)

    def nj_slot_activation(self, K, r, coeffs, mask_re, mask_im, act, stoc1, re, im, out, stream=None):
        cr, cm, co = re.c(), im.c(), out.c()
        cf = _coeffs(coeffs)
        _check(_lib.nj_slot_activation(self.ptr, int(K), int(r), None if cf is None else _np_ptr(cf),
                                       0 if cf is None else len(cf), None if mask_re is None else _dev_ptr(mask_re),
                                       None if mask_im is None else _dev_ptr(mask_im), int(act), stoc1.ptr,
                                       ctypes.byref(cr), ctypes.byref(cm), ctypes.byref(co), _stream(stream)),
               "nj_slot_activation")
        return out.sync_from(co)

    def nj_slot_activation_decompose(self, K, r, coeffs, mask_re, mask_im, act, dec_re, dec_im, stoc1, re, im, out,
                                     stream=None):
        cr, cm, co = re.c(), im.c(), out.c()
        cf = _coeffs(coeffs)
        _check(_lib.nj_slot_activation_decompose(
            self.ptr, int(K), int(r), None if cf is None else _np_ptr(cf), 0 if cf is None else len(cf),
            None if mask_re is None else _dev_ptr(mask_re), None if mask_im is None else _dev_ptr(mask_im), int(act),
            None if dec_re is None else dec_re.ptr, None if dec_im is None else dec_im.ptr, stoc1.ptr,
            ctypes.byref(cr), ctypes.byref(cm), ctypes.byref(co), _stream(stream)), "nj_slot_activation_decompose")
        return out.sync_from(co)

    def nj_conv_act_layer(self, conv, cts, K, r, coeffs, mask_re, mask_im, act, stoc1, ct, out, stream=None):
        ci, co = ct.c(), out.c()
        cf = _coeffs(coeffs)
        _check(_lib.nj_conv_act_layer(self.ptr, None if conv is None else conv.ptr, cts.ptr, int(K), int(r),
                                      None if cf is None else _np_ptr(cf), 0 if cf is None else len(cf),
                                      None if mask_re is None else _dev_ptr(mask_re),
                                      None if mask_im is None else _dev_ptr(mask_im), int(act), stoc1.ptr,
                                      ctypes.byref(ci), ctypes.byref(co), _stream(stream)), "nj_conv_act_layer")
        return out.sync_from(co)

    def nj_bootstrap(self, cts, K, r, coeffs, stoc1, ct, out, stream=None):
        ci, co = ct.c(), out.c()
        cf = _coeffs(coeffs)
        _check(_lib.nj_bootstrap(self.ptr, cts.ptr, int(K), int(r), None if cf is None else _np_ptr(cf),
                                 0 if cf is None else len(cf), stoc1.ptr, ctypes.byref(ci), ctypes.byref(co),
                                 _stream(stream)), "nj_bootstrap")
        return out.sync_from(co)

    def nj_timing_keys(self, pool):
        _check(_lib.nj_timing_keys(self.ptr, int(pool)), "nj_timing_keys")

    def nj_plan_create_random(self, level, u, offsets, n1=0, bi=1, bo=1, seed=1):
        off = np.ascontiguousarray(offsets, dtype=np.int32)
        h = vp()
        _check(_lib.nj_plan_create_random(self.ptr, int(level), int(u), _np_ptr(off), len(off), int(n1), int(bi),
                                          int(bo), u64(seed), ctypes.byref(h)), "nj_plan_create_random")
        return Plan(h)

    def nj_time_plan(self, plan, level, t=0, reps=3):
        ms = ctypes.c_float()
        _check(_lib.nj_time_plan(self.ptr, plan.ptr, int(t), int(level), int(reps), ctypes.byref(ms)),
               "nj_time_plan")
        return ms.value

    def nj_tune_split(self, plan, level, t=0, model=None, shortlist=3, reps=3, lazy=False):
        """(n1, hoist, lazy, ms, default ms) the library's autotuner picks for transform t;
        lazy=True also times the other giant-step ModDown form (else lazy is the plan's)"""
        n1, ho, lz = i32(), i32(), i32(-1)
        ms, dms = ctypes.c_float(), ctypes.c_float()
        _check(_lib.nj_tune_split(self.ptr, plan.ptr, int(t), int(level), model.ptr if model is not None else None,
                                  int(shortlist), int(reps), ctypes.byref(n1), ctypes.byref(ho),
                                  ctypes.cast(ctypes.pointer(lz), vp) if lazy else None, ctypes.byref(ms),
                                  ctypes.byref(dms)), "nj_tune_split")
        return n1.value, bool(ho.value), (bool(lz.value) if lazy else None), ms.value, dms.value

    def nj_cts_plan_create(self, groups):
        h = vp()
        _check(_lib.nj_cts_plan_create(self.ptr, groups, ctypes.byref(h)), "nj_cts_plan_create")
        return Plan(h)

    def nj_cts_plan_create_split(self, groups, n1s):
        n1 = np.ascontiguousarray(list(n1s), dtype=np.int32)
        assert n1.shape == (groups,)
        h = vp()
        _check(_lib.nj_cts_plan_create_split(self.ptr, int(groups), _np_ptr(n1), ctypes.byref(h)),
               "nj_cts_plan_create_split")
        return Plan(h)

    def cts_plan_from_spec(self, spec):
        """a CoeffToSlot plan from its description {"groups": d, "n1": [per group] (absent
        or null: the default split), "hoist": bool or [per group], "lazy": bool} - the
        form the learned plan is reported in, so it can be stored as JSON and rebuilt"""
        n1 = spec.get("n1")
        plan = self.nj_cts_plan_create_split(spec["groups"], n1) if n1 else self.nj_cts_plan_create(spec["groups"])
        plan.set_hoist(spec.get("hoist", True))
        return plan.set_lazy(spec.get("lazy", False))

    def decrypt_checked(self, ct, bound):
        """decrypted coefficients / scale (two limbs' CRT, one at level 0) and whether they
        are an unambiguous decryption of a message bounded by `bound`: false when the
        bound reaches half the modulus over the scale (values that large wrap around and
        cannot be told from small ones), or when a value exceeds the bound (the message
        outgrew it)"""
        k = min(2, ct.level + 1)
        d = self.torch.empty((ct.level + 1, self.N), dtype=self.torch.int64, device=self.device)
        self.nj_decrypt(ct, d)
        res = self.to_host(d)[:k]
        Q = 1
        for q in self.q[:k]:
            Q *= int(q)
        if k == 1:
            v = res[0].astype(np.float64)
            v[v > self.q[0] / 2] -= self.q[0]
        else:  # CRT of two limbs, centred
            q0, q1 = int(self.q[0]), int(self.q[1])
            inv = pow(q0, -1, q1)
            x = [int(a) + q0 * (((int(b) - int(a)) * inv) % q1) for a, b in zip(res[0], res[1])]
            v = np.array([float(t - Q) if t > Q // 2 else float(t) for t in x])
        v /= ct.scale
        return v, bool(bound < Q / (2.0 * ct.scale) and np.max(np.abs(v)) <= bound)

    def nj_cts_plan_features(self, groups, n1s=None, hoist=True):
        n1 = None if n1s is None else np.ascontiguousarray(list(n1s), dtype=np.int32)
        f = np.zeros((groups, 7), dtype=np.float32)
        _check(_lib.nj_cts_plan_features(self.ptr, int(groups), None if n1 is None else _np_ptr(n1), int(bool(hoist)),
                                         _np_ptr(f)), "nj_cts_plan_features")
        return f

    def nj_plan_set_diagonal(self, plan, t, idx, coeffs):
        cf = np.ascontiguousarray(coeffs, dtype=np.uint64)
        _check(_lib.nj_plan_set_diagonal(self.ptr, plan.ptr, t, idx, _np_ptr(cf)), "nj_plan_set_diagonal")

    def nj_plan_apply(self, plan, t, ct, out, hoist=1, stream=None):
        ci, co = ct.c(), out.c()
        _check(_lib.nj_plan_apply(self.ptr, plan.ptr, t, ctypes.byref(ci), ctypes.byref(co), int(hoist),
                                  _stream(stream)), "nj_plan_apply")
        return out.sync_from(co)

    def nj_conv2d_cins(self, plan, ct, out, stream=None):
        ci, co = ct.c(), out.c()
        _check(_lib.nj_conv2d_cins(self.ptr, plan.ptr, ctypes.byref(ci), ctypes.byref(co), _stream(stream)),
               "nj_conv2d_cins")
        return out.sync_from(co)

    def nj_coeff_to_slot(self, plan, ct, re, im, stream=None):
        ci, cr, cm = ct.c(), re.c(), im.c()
        _check(_lib.nj_coeff_to_slot(self.ptr, plan.ptr, ctypes.byref(ci), ctypes.byref(cr), ctypes.byref(cm),
                                     _stream(stream)), "nj_coeff_to_slot")
        re.sync_from(cr)
        im.sync_from(cm)
        return re, im
