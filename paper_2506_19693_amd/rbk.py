"""Thin ctypes binding of librbk (include/rbk.h).

Argument marshalling only: every operation runs in the HIP kernels of
librbk.so.  PyTorch supplies device memory (int64 tensors that hold the
uint64 residues bit for bit) and the current stream.  If the library is not
built, or no GPU is visible, calls fail loudly: there is no fallback.
"""
import atexit
import ctypes
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbk.so")

u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)
dblp = ctypes.POINTER(ctypes.c_double)
vp = ctypes.c_void_p
ci = ctypes.c_int
cu64 = ctypes.c_uint64


class RbkParams(ctypes.Structure):
    _fields_ = [
        ("log_n", ctypes.c_uint32),
        ("n_q", ctypes.c_uint32),
        ("q_bits", ctypes.POINTER(ctypes.c_uint32)),
        ("n_p", ctypes.c_uint32),
        ("p_bits", ctypes.POINTER(ctypes.c_uint32)),
        ("alpha", ctypes.c_uint32),
    ]


class RbkMlpDesc(ctypes.Structure):
    _fields_ = [
        ("k0", ctypes.c_uint32),
        ("n_layers", ctypes.c_uint32),
        ("widths", ctypes.POINTER(ctypes.c_uint32)),
        ("n_out", ctypes.c_uint32),
        ("r", ctypes.c_uint32),
        ("c", ctypes.c_uint32),
        ("act", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("log2_scale", ctypes.c_double),
        ("flags", ctypes.c_uint32),
    ]


MLP_LITERAL_DERIV = 1
MLP_L2_DECAY = 2
MLP_NO_BOOTSTRAP = 1
MLP_PER_SAMPLE = 2
MLP_SEQUENTIAL = 4


class RbkJob(ctypes.Structure):
    _fields_ = [
        ("kind", ci),
        ("tenant", ci),
        ("count", ci),
        ("level", ci),
        ("in_level", ci),
        ("d_a", vp),
        ("d_b", vp),
        ("d_out", vp),
        ("scales_in", dblp),
        ("scales_out", dblp),
        ("mlp", vp),
        ("d_x", vp),
        ("d_y_exp", vp),
        ("d_y_rep", vp),
        ("b", ci),
        ("scale", ctypes.c_double),
        ("t0", ci),
    ]


class RbkJobResult(ctypes.Structure):
    _fields_ = [
        ("status", ci),
        ("latency_ms", ctypes.c_double),
        ("queue_ms", ctypes.c_double),
        ("run_ms", ctypes.c_double),
        ("batch_cts", ci),
    ]


JOB_MULT_RESCALE = 1
JOB_BOOTSTRAP = 2
JOB_TRAIN_STEP = 3


class RbkBootParams(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_uint32),
        ("degree", ctypes.c_uint32),
        ("double_angle", ctypes.c_uint32),
        ("cts_levels", ctypes.c_uint32),
        ("stc_levels", ctypes.c_uint32),
        ("log2_rho", ctypes.c_uint32),
    ]


class RbkMrItem(ctypes.Structure):
    _fields_ = [
        ("ctx", ctypes.c_void_p),
        ("d_a", ctypes.c_void_p),
        ("d_b", ctypes.c_void_p),
        ("d_out", ctypes.c_void_p),
        ("level", ctypes.c_int),
        ("pad", ctypes.c_int),
    ]


class RbkNttItem(ctypes.Structure):
    _fields_ = [
        ("ctx", ctypes.c_void_p),
        ("d_limb", ctypes.c_void_p),
        ("prime", ctypes.c_int),
        ("pad", ctypes.c_int),
    ]


# name -> (restype, argtypes); the declarations of include/rbk.h
SIGNATURES = {
    "rbk_ctx_create": (ci, [ctypes.POINTER(RbkParams), ctypes.POINTER(vp)]),
    "rbk_ctx_destroy": (ci, [vp]),
    "rbk_set_stream": (ci, [vp, vp]),
    "rbk_sync": (ci, [vp]),
    "rbk_last_error": (ctypes.c_char_p, []),
    "rbk_moduli": (ci, [vp, u64p]),
    "rbk_psi": (ci, [vp, u64p]),
    "rbk_num_digits": (ci, [vp, ci]),
    "rbk_reserve": (ci, [vp, ci, ci]),
    "rbk_ntt": (ci, [vp, vp, ci, ctypes.POINTER(ci), ci, ci]),
    "rbk_set_secret": (ci, [vp, i64p]),
    "rbk_keygen_public": (ci, [vp, u64p, i64p]),
    "rbk_keygen_relin": (ci, [vp, u64p, i64p]),
    "rbk_keygen_galois": (ci, [vp, cu64, u64p, i64p]),
    "rbk_galois_elt": (cu64, [vp, ctypes.c_int64]),
    "rbk_key_export": (ci, [vp, cu64, u64p]),
    "rbk_keygen": (ci, [vp, cu64, ci, i64p, ci, ci]),
    "rbk_encrypt_seeded": (ci, [vp, vp, ci, cu64, cu64, vp]),
    "rbk_gauss_table": (ci, [u64p]),
    "rbk_ct_export": (ci, [vp, vp, ci, ci, u64p]),
    "rbk_add_scaled": (ci, [vp, vp, ctypes.c_double, vp, ctypes.c_double, vp, ci, dblp]),
    "rbk_sub_scaled": (ci, [vp, vp, ctypes.c_double, vp, ctypes.c_double, vp, ci, dblp]),
    "rbk_add_plain_scaled": (ci, [vp, vp, ctypes.c_double, vp, ctypes.c_double, vp, ci, dblp]),
    "rbk_ct_import": (ci, [vp, u64p, ci, ci, vp]),
    "rbk_encode": (ci, [vp, dblp, dblp, ctypes.c_size_t, ci, ctypes.c_double, vp]),
    "rbk_decode": (ci, [vp, vp, ci, ctypes.c_double, dblp, dblp, ctypes.c_size_t]),
    "rbk_encrypt": (ci, [vp, vp, ci, i64p, i64p, i64p, vp]),
    "rbk_decrypt": (ci, [vp, vp, ci, vp]),
    "rbk_add": (ci, [vp, vp, vp, vp, ci, ci]),
    "rbk_sub": (ci, [vp, vp, vp, vp, ci, ci]),
    "rbk_neg": (ci, [vp, vp, vp, ci, ci]),
    "rbk_mul_poly": (ci, [vp, vp, vp, vp, ci, ci]),
    "rbk_mul_plain": (ci, [vp, vp, vp, vp, ci]),
    "rbk_add_plain": (ci, [vp, vp, vp, vp, ci]),
    "rbk_mul_scalar": (ci, [vp, vp, u64p, vp, ci, ci]),
    "rbk_add_scalar": (ci, [vp, vp, u64p, vp, ci]),
    "rbk_tensor": (ci, [vp, vp, vp, vp, ci]),
    "rbk_modup": (ci, [vp, vp, vp, ci]),
    "rbk_key_inner_product": (ci, [vp, vp, cu64, vp, ci]),
    "rbk_moddown": (ci, [vp, vp, vp, ci, ci]),
    "rbk_keyswitch": (ci, [vp, cu64, vp, vp, ci]),
    "rbk_mult_relin": (ci, [vp, vp, vp, vp, ci]),
    "rbk_rescale": (ci, [vp, vp, vp, ci]),
    "rbk_automorph": (ci, [vp, vp, vp, ci, ci, cu64]),
    "rbk_rotate": (ci, [vp, vp, vp, ci, ctypes.c_int64]),
    "rbk_conjugate": (ci, [vp, vp, vp, ci]),
    "rbk_rotate_hoisted": (ci, [vp, vp, i64p, ci, vp, ci]),
    "rbk_mult_relin_batch": (ci, [vp, vp, vp, vp, ci, ci]),
    "rbk_rescale_batch": (ci, [vp, vp, vp, ci, ci]),
    "rbk_rescale_batch_noalloc": (ci, [vp, vp, vp, ci, ci]),
    "rbk_ntt_list": (ci, [vp, ctypes.POINTER(RbkNttItem), ci, ci]),
    "rbk_mult_relin_rescale_list": (ci, [vp, vp, vp, vp, ctypes.POINTER(ci), ci]),
    "rbk_mult_relin_rescale_multi": (ci, [vp, ctypes.POINTER(RbkMrItem), ci]),
    "rbk_rotate_hoisted_batch": (ci, [vp, vp, i64p, ci, vp, ci, ci]),
    "rbk_rotate_add_batch": (ci, [vp, vp, vp, vp, ci, ci, ctypes.c_int64]),
    "rbk_boot_setup": (ci, [vp, ctypes.POINTER(RbkBootParams)]),
    "rbk_boot_rotations": (ci, [vp, i64p, ci]),
    "rbk_boot_info": (ci, [vp, ctypes.POINTER(ci), ctypes.POINTER(ci), ctypes.POINTER(ci)]),
    "rbk_boot_constant_levels": (ci, [vp, ctypes.POINTER(ci), ctypes.POINTER(ci)]),
    "rbk_boot_export": (ci, [vp, u64p, u64p]),
    "rbk_boot_import": (ci, [vp, u64p, u64p]),
    "rbk_bootstrap_batch": (ci, [vp, vp, dblp, vp, dblp, ci]),
    "rbk_bootstrap": (ci, [vp, vp, ctypes.c_double, vp, dblp]),
    "rbk_mlp_create": (ci, [vp, ctypes.POINTER(RbkMlpDesc), ctypes.POINTER(vp)]),
    "rbk_mlp_destroy": (ci, [vp]),
    "rbk_mlp_info": (ci, [vp, ctypes.POINTER(ci)]),
    "rbk_mlp_rotations": (ci, [vp, i64p, ci]),
    "rbk_mlp_set_state": (ci, [vp, ci, vp, ci, ctypes.c_double]),
    "rbk_mlp_get_state": (ci, [vp, ci, vp, ctypes.POINTER(ci), dblp]),
    "rbk_mlp_set_mask": (ci, [vp, ci, vp]),
    "rbk_mlp_train_step": (ci, [vp, vp, vp, vp, ci, ci, ctypes.c_double, ci, ctypes.c_uint32]),
    "rbk_mlp_scalars": (ci, [vp, i64p, ci]),
    "rbk_mlp_infer": (ci, [vp, vp, ci, ci, ctypes.c_double, ci, vp, ctypes.POINTER(ci), dblp]),
    "rbk_mlp_set_weights": (ci, [vp, ctypes.POINTER(dblp), ctypes.POINTER(dblp), ctypes.POINTER(dblp),
                                 ctypes.POINTER(dblp), ci, cu64]),
    "rbk_mlp_get_weights": (ci, [vp, ctypes.POINTER(dblp), ctypes.POINTER(dblp), ctypes.POINTER(dblp),
                                 ctypes.POINTER(dblp)]),
    "rbk_server_create": (ci, [ctypes.c_uint64, ci, ci, ctypes.POINTER(vp)]),
    "rbk_server_add_tenant": (ci, [vp, vp, ctypes.POINTER(ci)]),
    "rbk_server_start": (ci, [vp]),
    "rbk_server_submit": (ci, [vp, ctypes.POINTER(RbkJob), u64p]),
    "rbk_server_wait": (ci, [vp, ctypes.c_uint64, ctypes.POINTER(RbkJobResult)]),
    "rbk_server_drain": (ci, [vp]),
    "rbk_server_stats": (ci, [vp, u64p]),
    "rbk_server_destroy": (ci, [vp]),
    "rbk_server_set_cross_tenant": (ci, [vp, ci]),
    "rbk_server_cross_merged": (ci, [vp, u64p]),
    "rbk_autotune": (ci, [vp, ci, ci, ctypes.c_char_p, ctypes.POINTER(ci)]),
    "rbk_tune_get": (ci, [vp, ctypes.POINTER(ci)]),
    "rbk_tune_set": (ci, [vp, ctypes.POINTER(ci)]),
    "rbk_workspace_words": (ci, [vp, ci, ci, ci, ctypes.POINTER(ctypes.c_size_t)]),
    "rbk_set_workspace": (ci, [vp, vp, ctypes.c_size_t]),
    "rbk_capture_begin": (ci, [vp]),
    "rbk_capture_end": (ci, [vp, ctypes.POINTER(vp)]),
    "rbk_graph_launch": (ci, [vp]),
    "rbk_graph_destroy": (ci, [vp]),
    "rbk_set_lanes": (ci, [vp, ci]),
    "rbk_timer_enable": (ci, [vp, ci]),
    "rbk_timer_read": (ci, [vp, ci, dblp, u64p, dblp]),
    "rbk_timer_name": (ctypes.c_char_p, [ci]),
    "rbk_ks_stats": (ci, [vp, u64p, dblp]),
}

_LIB = None


def load():
    """Load librbk.so (built by paper_2506_19693_amd/build.py).  Raises if absent."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("librbk.so is not built: run python paper_2506_19693_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


class RbkError(RuntimeError):
    pass


def _check(rc):
    if rc < 0:
        raise RbkError("librbk error %d: %s" % (rc, load().rbk_last_error().decode()))
    return rc


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("librbk needs a ROCm GPU: torch.cuda.is_available() is False")
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _h_u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(u64p)


def _h_i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(i64p)


def to_device(arr):
    """uint64 numpy array -> int64 CUDA tensor with the same bits."""
    torch = _torch()
    a = np.ascontiguousarray(arr, dtype=np.uint64).view(np.int64)
    return torch.from_numpy(a.copy()).to("cuda")


def to_host(t):
    """int64 CUDA tensor -> uint64 numpy array with the same bits."""
    return t.detach().cpu().numpy().view(np.uint64)


_LIVE_SERVERS = weakref.WeakSet()
_LIVE_GRAPHS = weakref.WeakSet()
_LIVE_MLPS = weakref.WeakSet()
_LIVE_CONTEXTS = weakref.WeakSet()


@atexit.register
def _close_all():
    """Release library objects while the HIP runtime is still up (objects that
    survive until interpreter teardown would otherwise be freed after it)."""
    for v in list(_LIVE_SERVERS):
        v.close()
    for v in list(_LIVE_GRAPHS):
        v.close()
    for m in list(_LIVE_MLPS):
        m.close()
    for c in list(_LIVE_CONTEXTS):
        c.close()


def mult_relin_rescale_multi(host, jobs, outs=None):
    """jobs: [(context, a, b, level)] of ciphertexts from any contexts (device
    tensors [2][level+1][N]); one set of launches on host's stream.  Returns
    the outputs [2][level][N]."""
    if outs is None:
        outs = [ctx.empty_ct(lv - 1) for ctx, _, _, lv in jobs]
    arr = (RbkMrItem * len(jobs))(*[RbkMrItem(ctx.h, _ptr(a), _ptr(b), _ptr(o), lv, 0)
                                   for (ctx, a, b, lv), o in zip(jobs, outs)])
    _check(host.lib.rbk_mult_relin_rescale_multi(host.h, arr, len(jobs)))
    return outs


def gauss_table():
    """The cumulative table of the library's Gaussian sampler."""
    out = np.zeros(20, dtype=np.uint64)
    _check(load().rbk_gauss_table(out.ctypes.data_as(u64p)))
    return [int(x) for x in out]


class Context:
    """One librbk context: ring degree 2^log_n, Q chain of sizes q_bits,
    special primes p_bits, alpha primes per key-switching digit."""

    def __init__(self, log_n, q_bits, p_bits, alpha):
        torch = _torch()
        self.lib = load()
        self.log_n = int(log_n)
        self.N = 1 << self.log_n
        self.nQ = len(q_bits)
        self.nP = len(p_bits)
        self.alpha = int(alpha)
        self.L = self.nQ - 1
        qb = (ctypes.c_uint32 * max(1, len(q_bits)))(*q_bits)
        pb = (ctypes.c_uint32 * max(1, len(p_bits)))(*p_bits)
        prm = RbkParams(self.log_n, self.nQ, qb, self.nP, pb, self.alpha)
        h = vp()
        _check(self.lib.rbk_ctx_create(ctypes.byref(prm), ctypes.byref(h)))
        self.h = h
        self.set_stream(torch.cuda.current_stream())
        m = np.zeros(self.nQ + self.nP, dtype=np.uint64)
        _check(self.lib.rbk_moduli(self.h, m.ctypes.data_as(u64p)))
        self.moduli = [int(x) for x in m]
        p = np.zeros(self.nQ + self.nP, dtype=np.uint64)
        _check(self.lib.rbk_psi(self.h, p.ctypes.data_as(u64p)))
        self.psi = [int(x) for x in p]
        self.beta = self.num_digits(self.L)
        self._deps = weakref.WeakSet()
        _LIVE_CONTEXTS.add(self)

    def close(self):
        # objects built on this context (MLPs) must go first: their destructors use it
        for dep in list(getattr(self, "_deps", ())):
            dep.close()
        if getattr(self, "h", None):
            self.lib.rbk_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- misc
    def set_stream(self, stream):
        _check(self.lib.rbk_set_stream(self.h, vp(stream.cuda_stream)))

    def sync(self):
        _check(self.lib.rbk_sync(self.h))

    def num_digits(self, level):
        return _check(self.lib.rbk_num_digits(self.h, level))

    def reserve(self, level, count):
        _check(self.lib.rbk_reserve(self.h, level, count))

    def empty(self, *shape):
        torch = _torch()
        return torch.empty(shape, dtype=torch.int64, device="cuda")

    def empty_ct(self, level, count=None):
        if count is None:
            return self.empty(2, level + 1, self.N)
        return self.empty(count, 2, level + 1, self.N)

    def ntt(self, t, prime_idx, inverse=False):
        """In-place NTT of t viewed as [count][len(prime_idx)][N]."""
        nl = len(prime_idx)
        count = t.numel() // (nl * self.N)
        idx = (ci * nl)(*prime_idx)
        _check(self.lib.rbk_ntt(self.h, _ptr(t), count, idx, nl, 1 if inverse else 0))
        return t

    def to_ntt(self, arr, level):
        """Host coefficient-domain residues [..][level+1][N] -> device NTT domain."""
        t = to_device(arr)
        return self.ntt(t, list(range(level + 1)))

    def to_coef(self, t, level):
        """Device NTT-domain residues [..][level+1][N] -> host coefficient domain."""
        c = t.clone()
        self.ntt(c, list(range(level + 1)), inverse=True)
        return to_host(c)

    # ---------------------------------------------------------------- keys
    def set_secret(self, s):
        s, ps = _h_i64(s)
        _check(self.lib.rbk_set_secret(self.h, ps))

    def keygen_public(self, a, e):
        a, pa = _h_u64(a)
        e, pe = _h_i64(e)
        _check(self.lib.rbk_keygen_public(self.h, pa, pe))

    def keygen_relin(self, a, e):
        a, pa = _h_u64(a)
        e, pe = _h_i64(e)
        _check(self.lib.rbk_keygen_relin(self.h, pa, pe))

    def keygen_galois(self, g, a, e):
        a, pa = _h_u64(a)
        e, pe = _h_i64(e)
        _check(self.lib.rbk_keygen_galois(self.h, int(g), pa, pe))

    def galois_elt(self, k):
        return int(self.lib.rbk_galois_elt(self.h, int(k)))

    def galois_conj(self):
        return 2 * self.N - 1

    def key_export(self, g=0):
        out = np.zeros((self.beta, 2, self.nQ + self.nP, self.N), dtype=np.uint64)
        _check(self.lib.rbk_key_export(self.h, int(g), out.ctypes.data_as(u64p)))
        return out

    def keygen(self, seed, secret_hw=0, rot_steps=(), conj=False):
        """Secret, public, relinearisation and Galois keys drawn in the library from `seed`."""
        ks = np.ascontiguousarray(list(rot_steps) or [0], dtype=np.int64)
        _check(self.lib.rbk_keygen(self.h, int(seed), int(secret_hw), ks.ctypes.data_as(i64p), len(rot_steps),
                                   1 if conj else 0))

    def encrypt_seeded(self, pt, level, seed, index):
        ct = self.empty_ct(level)
        _check(self.lib.rbk_encrypt_seeded(self.h, _ptr(pt), level, int(seed), int(index), _ptr(ct)))
        return ct

    def ct_export(self, t, level):
        """Device NTT-domain polynomials [npoly][level+1][N] -> host coefficient domain."""
        npoly = self._npoly(t, level)
        out = np.zeros(tuple(t.shape), dtype=np.uint64)
        _check(self.lib.rbk_ct_export(self.h, _ptr(t), level, npoly, out.ctypes.data_as(u64p)))
        return out

    def ct_import(self, arr, level):
        """Host coefficient-domain residues [npoly][level+1][N] -> device NTT domain."""
        a, pa = _h_u64(arr)
        npoly = a.size // ((level + 1) * self.N)
        t = self.empty(*a.shape)
        _check(self.lib.rbk_ct_import(self.h, pa, level, npoly, _ptr(t)))
        return t

    # ---------------------------------------------------------------- encoding
    def encode(self, z, level, scale):
        z = np.asarray(z)
        re = np.ascontiguousarray(z.real, dtype=np.float64)
        im = np.ascontiguousarray(z.imag, dtype=np.float64) if np.iscomplexobj(z) else None
        pt = self.empty(level + 1, self.N)
        _check(self.lib.rbk_encode(self.h, re.ctypes.data_as(dblp), im.ctypes.data_as(dblp) if im is not None else None,
                                   len(re), level, float(scale), _ptr(pt)))
        return pt

    def decode(self, pt, level, scale, n=None):
        n = self.N // 2 if n is None else n
        re = np.zeros(n)
        im = np.zeros(n)
        _check(self.lib.rbk_decode(self.h, _ptr(pt), level, float(scale), re.ctypes.data_as(dblp), im.ctypes.data_as(dblp), n))
        return re + 1j * im

    def encrypt(self, pt, level, v, e0, e1):
        v, pv = _h_i64(v)
        e0, p0 = _h_i64(e0)
        e1, p1 = _h_i64(e1)
        ct = self.empty_ct(level)
        _check(self.lib.rbk_encrypt(self.h, _ptr(pt), level, pv, p0, p1, _ptr(ct)))
        return ct

    def decrypt(self, ct, level):
        pt = self.empty(level + 1, self.N)
        _check(self.lib.rbk_decrypt(self.h, _ptr(ct), level, _ptr(pt)))
        return pt

    # ---------------------------------------------------------------- ring ops
    def _npoly(self, t, level):
        return t.numel() // ((level + 1) * self.N)

    def add(self, a, b, level):
        out = self.empty(*a.shape)
        _check(self.lib.rbk_add(self.h, _ptr(a), _ptr(b), _ptr(out), level, self._npoly(a, level)))
        return out

    def sub(self, a, b, level):
        out = self.empty(*a.shape)
        _check(self.lib.rbk_sub(self.h, _ptr(a), _ptr(b), _ptr(out), level, self._npoly(a, level)))
        return out

    def _scaled(self, fn, a, sa, b, sb, level):
        out = self.empty(*a.shape)
        so = ctypes.c_double()
        _check(fn(self.h, _ptr(a), float(sa), _ptr(b), float(sb), _ptr(out), level, ctypes.byref(so)))
        return out, so.value

    def add_scaled(self, a, sa, b, sb, level):
        """(a + b, scale); RbkError (RBK_ESCALE) unless the scales agree to 2^-30."""
        return self._scaled(self.lib.rbk_add_scaled, a, sa, b, sb, level)

    def sub_scaled(self, a, sa, b, sb, level):
        return self._scaled(self.lib.rbk_sub_scaled, a, sa, b, sb, level)

    def add_plain_scaled(self, ct, sct, pt, spt, level):
        return self._scaled(self.lib.rbk_add_plain_scaled, ct, sct, pt, spt, level)

    def neg(self, a, level):
        out = self.empty(*a.shape)
        _check(self.lib.rbk_neg(self.h, _ptr(a), _ptr(out), level, self._npoly(a, level)))
        return out

    def mul_poly(self, a, b, level):
        out = self.empty(*a.shape)
        _check(self.lib.rbk_mul_poly(self.h, _ptr(a), _ptr(b), _ptr(out), level, self._npoly(a, level)))
        return out

    def mul_plain(self, ct, pt, level):
        out = self.empty_ct(level)
        _check(self.lib.rbk_mul_plain(self.h, _ptr(ct), _ptr(pt), _ptr(out), level))
        return out

    def add_plain(self, ct, pt, level):
        out = self.empty_ct(level)
        _check(self.lib.rbk_add_plain(self.h, _ptr(ct), _ptr(pt), _ptr(out), level))
        return out

    def mul_scalar(self, a, scal, level):
        s, ps = _h_u64(scal)
        out = self.empty(*a.shape)
        _check(self.lib.rbk_mul_scalar(self.h, _ptr(a), ps, _ptr(out), level, self._npoly(a, level)))
        return out

    def add_scalar(self, ct, scal, level):
        s, ps = _h_u64(scal)
        out = self.empty_ct(level)
        _check(self.lib.rbk_add_scalar(self.h, _ptr(ct), ps, _ptr(out), level))
        return out

    def tensor(self, a, b, level):
        out = self.empty(3, level + 1, self.N)
        _check(self.lib.rbk_tensor(self.h, _ptr(a), _ptr(b), _ptr(out), level))
        return out

    # ---------------------------------------------------------------- key switching
    def modup(self, d, level):
        E = level + 1 + self.nP
        out = self.empty(self.num_digits(level), E, self.N)
        _check(self.lib.rbk_modup(self.h, _ptr(d), _ptr(out), level))
        return out

    def key_inner_product(self, ext, g, level):
        E = level + 1 + self.nP
        out = self.empty(2, E, self.N)
        _check(self.lib.rbk_key_inner_product(self.h, _ptr(ext), int(g), _ptr(out), level))
        return out

    def moddown(self, u, level):
        E = level + 1 + self.nP
        npoly = u.numel() // (E * self.N)
        out = self.empty(npoly, level + 1, self.N)
        _check(self.lib.rbk_moddown(self.h, _ptr(u), _ptr(out), level, npoly))
        return out

    def keyswitch(self, g, d, level):
        out = self.empty_ct(level)
        _check(self.lib.rbk_keyswitch(self.h, int(g), _ptr(d), _ptr(out), level))
        return out

    def mult_relin(self, a, b, level):
        out = self.empty_ct(level)
        _check(self.lib.rbk_mult_relin(self.h, _ptr(a), _ptr(b), _ptr(out), level))
        return out

    def rescale(self, ct, level):
        out = self.empty_ct(level - 1)
        _check(self.lib.rbk_rescale(self.h, _ptr(ct), _ptr(out), level))
        return out

    def automorph(self, t, g, level):
        out = self.empty(*t.shape)
        _check(self.lib.rbk_automorph(self.h, _ptr(t), _ptr(out), level, self._npoly(t, level), int(g)))
        return out

    def rotate(self, ct, k, level):
        out = self.empty_ct(level)
        _check(self.lib.rbk_rotate(self.h, _ptr(ct), _ptr(out), level, int(k)))
        return out

    def conjugate(self, ct, level):
        out = self.empty_ct(level)
        _check(self.lib.rbk_conjugate(self.h, _ptr(ct), _ptr(out), level))
        return out

    def rotate_hoisted(self, ct, ks, level):
        ks_a, pk = _h_i64(ks)
        out = self.empty(len(ks), 2, level + 1, self.N)
        _check(self.lib.rbk_rotate_hoisted(self.h, _ptr(ct), pk, len(ks), _ptr(out), level))
        return out

    # ---------------------------------------------------------------- bootstrapping
    def boot_setup(self, K=23, degree=59, double_angle=2, cts_levels=3, stc_levels=3, log2_rho=2):
        prm = RbkBootParams(K, degree, double_angle, cts_levels, stc_levels, log2_rho)
        _check(self.lib.rbk_boot_setup(self.h, ctypes.byref(prm)))
        self.boot_levels, self.boot_nplain, self.boot_nscalar = self.boot_info()

    def boot_rotations(self):
        n = _check(self.lib.rbk_boot_rotations(self.h, None, 0))
        ks = np.zeros(max(n, 1), dtype=np.int64)
        _check(self.lib.rbk_boot_rotations(self.h, ks.ctypes.data_as(i64p), n))
        return [int(k) for k in ks[:n]]

    def boot_info(self):
        lv = (ci * 4)()
        npl, nsc = ci(), ci()
        _check(self.lib.rbk_boot_info(self.h, lv, ctypes.byref(npl), ctypes.byref(nsc)))
        return list(lv), npl.value, nsc.value

    def boot_constant_levels(self):
        _, npl, nsc = self.boot_info()
        pl = (ci * max(npl, 1))()
        sl = (ci * max(nsc, 1))()
        _check(self.lib.rbk_boot_constant_levels(self.h, pl, sl))
        return list(pl)[:npl], list(sl)[:nsc]

    def boot_export(self):
        pl, sl = self.boot_constant_levels()
        P = np.zeros(sum((l + 1) * self.N for l in pl), dtype=np.uint64)
        S = np.zeros(max(1, sum(l + 1 for l in sl)), dtype=np.uint64)
        _check(self.lib.rbk_boot_export(self.h, P.ctypes.data_as(u64p), S.ctypes.data_as(u64p)))
        plains, scal, o = [], [], 0
        for l in pl:
            plains.append(P[o: o + (l + 1) * self.N].reshape(l + 1, self.N))
            o += (l + 1) * self.N
        o = 0
        for l in sl:
            scal.append(S[o: o + l + 1])
            o += l + 1
        return plains, scal

    def boot_import(self, plains, scalars):
        P = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.uint64).ravel() for p in plains]))
        S = np.ascontiguousarray(np.concatenate([np.asarray(s, dtype=np.uint64).ravel() for s in scalars]))
        _check(self.lib.rbk_boot_import(self.h, P.ctypes.data_as(u64p), S.ctypes.data_as(u64p)))

    def bootstrap_batch(self, cts, scales, out=None):
        """cts: [count][2][1][N] level-0 ciphertexts; returns (outputs, scales)."""
        count = cts.shape[0]
        lo = self.boot_levels[3]
        out = self.empty_ct(lo, count) if out is None else out
        sc = np.ascontiguousarray(scales, dtype=np.float64)
        so = np.zeros(count)
        _check(self.lib.rbk_bootstrap_batch(self.h, _ptr(cts), sc.ctypes.data_as(dblp), _ptr(out),
                                            so.ctypes.data_as(dblp), count))
        return out, so

    def bootstrap(self, ct, scale):
        lo = self.boot_levels[3]
        out = self.empty_ct(lo)
        so = ctypes.c_double()
        _check(self.lib.rbk_bootstrap(self.h, _ptr(ct), float(scale), _ptr(out), ctypes.byref(so)))
        return out, so.value

    # ---------------------------------------------------------------- workspace
    def workspace_words(self, level, count, n_rot=0):
        """Words of workspace batched calls on count ciphertexts at level need
        (mult_relin, rescale, a hoisted batch of n_rot rotations)."""
        w = ctypes.c_size_t()
        _check(self.lib.rbk_workspace_words(self.h, level, count, n_rot, ctypes.byref(w)))
        return w.value

    def set_workspace(self, buf):
        """Use the device tensor buf (int64, kept alive by this object) as the
        context's workspace; None returns to a library-owned one."""
        if buf is None:
            _check(self.lib.rbk_set_workspace(self.h, None, 0))
        else:
            _check(self.lib.rbk_set_workspace(self.h, _ptr(buf), buf.numel()))
        self._ws_buf = buf

    # ---------------------------------------------------------------- autotuner
    def autotune(self, level, count, cache_path=None):
        """Time the NTT split, the NTT chunk and the inner-product chunk on
        (level, count); returns {"logC": .., "cpc": .., "chunk": ..} now in force."""
        cfg = (ci * 3)()
        path = cache_path.encode() if cache_path else None
        _check(self.lib.rbk_autotune(self.h, level, count, path, cfg))
        return {"logC": cfg[0], "cpc": cfg[1], "chunk": cfg[2]}

    def tune_get(self):
        cfg = (ci * 3)()
        _check(self.lib.rbk_tune_get(self.h, cfg))
        return {"logC": cfg[0], "cpc": cfg[1], "chunk": cfg[2]}

    def tune_set(self, logC, cpc, chunk=None):
        if chunk is None:
            chunk = self.tune_get()["chunk"]
        _check(self.lib.rbk_tune_set(self.h, (ci * 3)(logC, cpc, chunk)))

    # ---------------------------------------------------------------- graph capture
    def capture(self, fn):
        """Capture the library work of fn() into a Graph.  fn must have run
        once eagerly before (buffers sized); it runs on a side stream while
        capturing, and nothing executes until the graph is launched."""
        torch = _torch()
        side = torch.cuda.Stream()
        torch.cuda.synchronize()
        self.set_stream(side)
        h = vp()
        try:
            _check(self.lib.rbk_capture_begin(self.h))
            try:
                fn()
            except BaseException:
                if self.lib.rbk_capture_end(self.h, ctypes.byref(h)) == 0 and h:
                    self.lib.rbk_graph_destroy(h)
                raise
            _check(self.lib.rbk_capture_end(self.h, ctypes.byref(h)))
        finally:
            self.set_stream(torch.cuda.current_stream())
        return Graph(self, h, side)

    # ---------------------------------------------------------------- lanes
    def set_lanes(self, n):
        """Side streams (lanes, 1..3) for hoisted-rotation ModDowns, bootstrap
        giant steps and EvalMod products; 1 runs everything on the context
        stream.  Not used while timers run or while the stream is captured."""
        _check(self.lib.rbk_set_lanes(self.h, int(n)))

    # ---------------------------------------------------------------- timers
    def timer_enable(self, on=True):
        _check(self.lib.rbk_timer_enable(self.h, 1 if on else 0))

    def ks_stats(self):
        """(key switches, method bytes) since the last timer_enable."""
        n, b = ctypes.c_uint64(), ctypes.c_double()
        _check(self.lib.rbk_ks_stats(self.h, ctypes.byref(n), ctypes.byref(b)))
        return n.value, b.value

    def timer_read(self):
        """{kernel name: (ms, launches, algorithmic bytes)} of every timed kernel."""
        out = {}
        cls = 0
        while True:
            name = self.lib.rbk_timer_name(cls)
            if name is None:
                break
            ms, bts = ctypes.c_double(), ctypes.c_double()
            n = ctypes.c_uint64()
            _check(self.lib.rbk_timer_read(self.h, cls, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(bts)))
            if n.value:
                out[name.decode()] = (ms.value, n.value, bts.value)
            cls += 1
        return out

    # ---------------------------------------------------------------- batched
    def mult_relin_batch(self, a, b, level, out=None):
        count = a.shape[0]
        out = self.empty_ct(level, count) if out is None else out
        _check(self.lib.rbk_mult_relin_batch(self.h, _ptr(a), _ptr(b), _ptr(out), level, count))
        return out

    def rescale_batch(self, ct, level, out=None):
        count = ct.shape[0]
        out = self.empty_ct(level - 1, count) if out is None else out
        _check(self.lib.rbk_rescale_batch(self.h, _ptr(ct), _ptr(out), level, count))
        return out

    def rescale_batch_noalloc(self, ct, level, out):
        """rescale_batch with the library's fixed scratch array (no device
        allocation; out must be given)."""
        count = ct.shape[0]
        _check(self.lib.rbk_rescale_batch_noalloc(self.h, _ptr(ct), _ptr(out), level, count))
        return out

    def mult_relin_rescale_list(self, a, b, levels, out=None):
        """Uneven levels in one batch: a, b [count][2][Lm+1][N] with ciphertext
        i in limbs 0..levels[i]; returns [count][2][Lm][N] with ciphertext i's
        rescaled product in limbs 0..levels[i]-1."""
        count = a.shape[0]
        Lm = max(levels)
        if len(levels) != count or a.shape[2] != Lm + 1 or b.shape != a.shape:
            raise ValueError("a, b must be [count][2][max(levels)+1][N]")
        out = self.empty_ct(Lm - 1, count) if out is None else out
        lv = (ci * count)(*[int(x) for x in levels])
        _check(self.lib.rbk_mult_relin_rescale_list(self.h, _ptr(a), _ptr(b), _ptr(out), lv, count))
        return out

    def ntt_list(self, items, inverse=False):
        """In-place NTT of a list of limbs: items = [(ctx, tensor, offset, prime)],
        the limb being the N residues of ctx's ring at tensor's element offset;
        launched on this context's stream."""
        arr = (RbkNttItem * len(items))()
        for k, (ctx, t, off, prime) in enumerate(items):
            if t.dtype.itemsize != 8 or off < 0 or off + ctx.N > t.numel():
                raise ValueError("limb outside its tensor")
            arr[k] = RbkNttItem(ctx.h, t.data_ptr() + 8 * off, int(prime), 0)
        _check(self.lib.rbk_ntt_list(self.h, arr, len(items), 1 if inverse else 0))

    def rotate_add_batch(self, ct, k, add, level, out=None):
        """add + Rot(ct, k) for [count][2][l+1][N] batches (add may be ct or out)."""
        count = ct.shape[0]
        out = self.empty(count, 2, level + 1, self.N) if out is None else out
        _check(self.lib.rbk_rotate_add_batch(self.h, _ptr(ct), _ptr(add), _ptr(out), level, count, int(k)))
        return out

    def rotate_hoisted_batch(self, ct, ks, level, out=None):
        count = ct.shape[0]
        ks_a, pk = _h_i64(ks)
        out = self.empty(count, len(ks), 2, level + 1, self.N) if out is None else out
        _check(self.lib.rbk_rotate_hoisted_batch(self.h, _ptr(ct), pk, len(ks), _ptr(out), level, count))
        return out


class Graph:
    """A captured sequence of library calls (rbk_capture_*); launch() replays
    it on the context's current stream."""

    def __init__(self, ctx, h, side):
        self.ctx = ctx
        self.lib = ctx.lib
        self.h = h
        self._side = side
        _LIVE_GRAPHS.add(self)

    def launch(self):
        _check(self.lib.rbk_graph_launch(self.h))

    def close(self):
        if getattr(self, "h", None):
            self.lib.rbk_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The packed MLP training step of one context (rbk_mlp_* of rbk.h).

    widths: hidden widths k_1..k_H; act: (a1, a2, a3) of
    f(z) = a1 z + a2 z^2 + a3 z^3."""

    def __init__(self, ctx, k0, widths, n_out, r, c, act=(1.0, 1.0, 0.0), gamma=0.001, eta=0.001, mu=0.9,
                 log2_scale=50.0, literal_deriv=False, l2_decay=False):
        self.ctx = ctx
        self.lib = ctx.lib
        w = (ctypes.c_uint32 * len(widths))(*widths)
        flags = (MLP_LITERAL_DERIV if literal_deriv else 0) | (MLP_L2_DECAY if l2_decay else 0)
        self._w = w
        d = RbkMlpDesc(k0, len(widths), w, n_out, r, c, (ctypes.c_double * 3)(*act), gamma, eta, mu, log2_scale,
                       flags)
        h = vp()
        _check(self.lib.rbk_mlp_create(ctx.h, ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        info = (ci * 3)()
        _check(self.lib.rbk_mlp_info(self.h, info))
        self.tiles, self.n_state, self.depth = list(info)
        ctx._deps.add(self)
        _LIVE_MLPS.add(self)

    def close(self):
        if getattr(self, "h", None):
            self.lib.rbk_mlp_destroy(self.h)
            self.h = None
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rotations(self):
        n = _check(self.lib.rbk_mlp_rotations(self.h, None, 0))
        ks = np.zeros(max(n, 1), dtype=np.int64)
        _check(self.lib.rbk_mlp_rotations(self.h, ks.ctypes.data_as(i64p), n))
        return [int(k) for k in ks[:n]]

    def set_state(self, idx, ct, level, scale):
        _check(self.lib.rbk_mlp_set_state(self.h, idx, _ptr(ct), level, float(scale)))

    def get_state(self, idx, copy=True):
        """(ciphertext tensor or None, level, scale) of state slot idx."""
        lv, sc = ci(), ctypes.c_double()
        _check(self.lib.rbk_mlp_get_state(self.h, idx, None, ctypes.byref(lv), ctypes.byref(sc)))
        if not copy:
            return None, lv.value, sc.value
        out = self.ctx.empty_ct(lv.value)
        _check(self.lib.rbk_mlp_get_state(self.h, idx, _ptr(out), ctypes.byref(lv), ctypes.byref(sc)))
        return out, lv.value, sc.value

    def set_mask(self, level, pt):
        _check(self.lib.rbk_mlp_set_mask(self.h, level, _ptr(pt)))

    @staticmethod
    def _mats(ms):
        if ms is None:
            return None, None
        arrs = [np.ascontiguousarray(m, dtype=np.float64) for m in ms]
        return arrs, (dblp * len(arrs))(*[a.ctypes.data_as(dblp) for a in arrs])

    def set_weights(self, Ws, Wstars, Vs=None, Vstars=None, level=None, seed=1):
        """Float64 weights (and velocities) -> packed, encrypted state at `level` (default: top)."""
        level = self.ctx.L if level is None else level
        keep = [self._mats(m) for m in (Ws, Wstars, Vs, Vstars)]
        _check(self.lib.rbk_mlp_set_weights(self.h, keep[0][1], keep[1][1], keep[2][1], keep[3][1], level, int(seed)))

    def get_weights(self, dims, n_out, velocities=True):
        """Decrypted (Ws, Wstars, Vs, Vstars) for layer dims [(k_{h-1}, k_h)]."""
        Ws = [np.zeros(dk) for dk in dims]
        Wst = [np.zeros((dk[1], n_out)) for dk in dims]
        Vs = [np.zeros(dk) for dk in dims] if velocities else None
        Vst = [np.zeros((dk[1], n_out)) for dk in dims] if velocities else None
        ptrs = [self._mats(m)[1] for m in (Ws, Wst, Vs, Vst)]
        _check(self.lib.rbk_mlp_get_weights(self.h, *ptrs))
        return Ws, Wst, Vs, Vst

    def train_step(self, x, y_exp, y_rep, level, scale, t, bootstrap=True, per_sample=False, block_parallel=True):
        """x: [b][tiles][2][level+1][N], y_exp / y_rep: [b][2][level+1][N] device tensors.
        block_parallel=False keeps every block's backward pass on the context stream."""
        b = x.shape[0]
        flags = ((0 if bootstrap else MLP_NO_BOOTSTRAP) | (MLP_PER_SAMPLE if per_sample else 0)
                 | (0 if block_parallel else MLP_SEQUENTIAL))
        _check(self.lib.rbk_mlp_train_step(self.h, _ptr(x), _ptr(y_exp), _ptr(y_rep), b, level, float(scale), t,
                                           flags))

    def infer(self, x, level, scale, last):
        """Forward pass of blocks 1..last on x [b][tiles][2][level+1][N]; returns
        [(outputs [b][2][lv+1][N], lv, scale)] of each local classifier h <= last."""
        b = x.shape[0]
        out = self.ctx.empty(last, b, 2, level + 1, self.ctx.N)
        lv = (ci * last)()
        sc = (ctypes.c_double * last)()
        _check(self.lib.rbk_mlp_infer(self.h, _ptr(x), b, level, float(scale), last, _ptr(out), lv, sc))
        res = []
        for h in range(last):
            n = 2 * (lv[h] + 1) * self.ctx.N       # each output sits at the start of its slot
            res.append((out[h].reshape(b, -1)[:, :n].reshape(b, 2, lv[h] + 1, self.ctx.N).contiguous(), lv[h], sc[h]))
        return res

    def scalars(self):
        n = _check(self.lib.rbk_mlp_scalars(self.h, None, 0))
        out = np.zeros(max(n, 1), dtype=np.int64)
        _check(self.lib.rbk_mlp_scalars(self.h, out.ctypes.data_as(i64p), n))
        return [int(v) for v in out[:n]]


class Server:
    """The serving loop of rbk.h (rbk_server_*).  Tensors named by a job are
    kept referenced here until the job is waited for."""

    def __init__(self, hbm_budget, max_batch=64, max_boot_batch=16):
        self.lib = load()
        h = vp()
        _check(self.lib.rbk_server_create(int(hbm_budget), int(max_batch), int(max_boot_batch), ctypes.byref(h)))
        self.h = h
        self._keep = {}
        self.tenants = []
        _LIVE_SERVERS.add(self)

    def add_tenant(self, ctx):
        t = ci()
        _check(self.lib.rbk_server_add_tenant(self.h, ctx.h, ctypes.byref(t)))
        self.tenants.append(ctx)
        return t.value

    def start(self):
        _check(self.lib.rbk_server_start(self.h))

    def _submit(self, job, keep):
        jid = ctypes.c_uint64()
        _check(self.lib.rbk_server_submit(self.h, ctypes.byref(job), ctypes.byref(jid)))
        self._keep[jid.value] = keep
        return jid.value

    def submit_mult(self, tenant, a, b, level, out, in_level=None):
        """out[i] = Rescale(mult_relin(a[i], b[i])) at `level`; a, b: [count][2][in_level+1][N]."""
        in_level = level if in_level is None else in_level
        j = RbkJob(kind=JOB_MULT_RESCALE, tenant=tenant, count=a.shape[0], level=level, in_level=in_level,
                   d_a=a.data_ptr(), d_b=b.data_ptr(), d_out=out.data_ptr())
        return self._submit(j, (a, b, out))

    def submit_bootstrap(self, tenant, cts, scales, out, in_level=0):
        """out[i] = Bootstrap(cts[i]); returns (id, host array the output scales are written to)."""
        sc = np.ascontiguousarray(scales, dtype=np.float64)
        so = np.zeros(len(sc))
        j = RbkJob(kind=JOB_BOOTSTRAP, tenant=tenant, count=len(sc), level=0, in_level=in_level,
                   d_a=cts.data_ptr(), d_out=out.data_ptr(), scales_in=sc.ctypes.data_as(dblp),
                   scales_out=so.ctypes.data_as(dblp))
        return self._submit(j, (cts, out, sc, so)), so

    def submit_train(self, tenant, mlp, x, y_exp, y_rep, level, scale, t0, steps=1):
        j = RbkJob(kind=JOB_TRAIN_STEP, tenant=tenant, count=steps, level=level, in_level=level, mlp=mlp.h,
                   d_x=x.data_ptr(), d_y_exp=y_exp.data_ptr(), d_y_rep=y_rep.data_ptr(), b=x.shape[0],
                   scale=float(scale), t0=t0)
        return self._submit(j, (mlp, x, y_exp, y_rep))

    def wait(self, jid):
        r = RbkJobResult()
        rc = self.lib.rbk_server_wait(self.h, jid, ctypes.byref(r))
        self._keep.pop(jid, None)
        _check(rc)
        return {"latency_ms": r.latency_ms, "queue_ms": r.queue_ms, "run_ms": r.run_ms, "batch_cts": r.batch_cts}

    def drain(self):
        _check(self.lib.rbk_server_drain(self.h))

    def set_cross_tenant(self, on=True):
        _check(self.lib.rbk_server_set_cross_tenant(self.h, 1 if on else 0))

    def stats(self):
        st = np.zeros(6, dtype=np.uint64)
        _check(self.lib.rbk_server_stats(self.h, st.ctypes.data_as(u64p)))
        keys = ["jobs_done", "batches", "jobs_merged", "ledger_peak", "ledger_now", "budget"]
        out = {k: int(v) for k, v in zip(keys, st)}
        n = ctypes.c_uint64()
        _check(self.lib.rbk_server_cross_merged(self.h, ctypes.byref(n)))
        out["jobs_cross_tenant"] = int(n.value)
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.rbk_server_destroy(self.h)
            self.h = None
        self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
