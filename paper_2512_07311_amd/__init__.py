"""Python binding of librcs (ctypes): argument marshalling only.

Every computation runs in the HIP library; torch is used for device memory
(tensor storage passed as raw pointers) and streams.  Importing this module
fails loudly when librcs.so has not been built: there is no CPU fallback.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librcs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("librcs.so is not built (run __graft_entry__.build() or "
                      "python paper_2512_07311_amd/build_lib.py)")
# torch ships its own HIP runtime; loading it first makes librcs bind to the
# same runtime (two runtimes in one process do not share devices or streams)
try:
    import torch as _torch  # noqa: F401
except ImportError:
    _torch = None
_lib = C.CDLL(LIB_PATH)

RCS_PREC_C128, RCS_PREC_C64, RCS_PREC_SPLIT_BF16 = 0, 1, 2
RCS_RANK_FULL_SVD, RCS_RANK_LEARNED, RCS_RANK_RSVD_AT_CAP = 0, 1, 2
PRECISIONS = {"c128": 0, "c64": 1, "split_bf16": 2}
SVD_PRECISIONS = {"f64": 0, "f32": 1}
NETWORKS = {"snake": 0, "interleaved": 1}
LATTICES = {"rect": 0, "rotated": 1}
MLP_PARAMS = 66 * 128 + 128 + 128 * 128 + 128 + 128 * 32 + 32

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "OUT_OF_MEMORY",
          4: "DEVICE", 5: "NUMERIC", 6: "STATE"}


class RcsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class CircuitDesc(C.Structure):
    _fields_ = [("rows", C.c_int32), ("cols", C.c_int32), ("n_cycles", C.c_int32),
                ("seed", C.c_uint64), ("n_removed", C.c_int32),
                ("removed_sites", C.POINTER(C.c_int32)), ("n_removed_random", C.c_int32),
                ("pattern", C.c_char_p), ("theta", C.c_double), ("phi", C.c_double),
                ("final_1q_layer", C.c_int32), ("swap_network", C.c_int32), ("lattice", C.c_int32)]


class BuildOpts(C.Structure):
    _fields_ = [("contraction", C.c_int32), ("rank_mode", C.c_int32),
                ("fallback_tau", C.c_double), ("mlp_weights_host", C.POINTER(C.c_float)),
                ("mlp_count", C.c_int64), ("rsvd_oversample", C.c_int32),
                ("rsvd_power_iters", C.c_int32), ("rsvd_seed", C.c_uint64),
                ("stream", C.c_void_p), ("log_spectra", C.c_int32), ("max_ops", C.c_int32),
                ("canonicalize", C.c_int32), ("svd_precision", C.c_int32)]


class StateInfo(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("max_bond", C.c_int32), ("center", C.c_int32),
                ("canonical", C.c_int32), ("n_truncations", C.c_int32),
                ("n_fallbacks", C.c_int32), ("n_rsvd_accepted", C.c_int32),
                ("jacobi_sweeps_max", C.c_int32), ("log_fidelity_est", C.c_double),
                ("sum_eps", C.c_double), ("build_seconds", C.c_double),
                ("svd_seconds", C.c_double), ("device_bytes", C.c_int64),
                ("n_center_moves", C.c_int32), ("nominal_svd_flops", C.c_double),
                ("nominal_qr_flops", C.c_double), ("n_precond", C.c_int32),
                ("n_precond_fallback", C.c_int32), ("n_center_moves_cholqr", C.c_int32),
                ("n_svd_f32", C.c_int32), ("n_svd_f32_redone", C.c_int32)]


_vp, _i32, _i64, _u64, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
_P = C.POINTER
_SIGS = {
    "rcs_circuit_create": [_P(CircuitDesc), _P(_vp)],
    "rcs_circuit_info": [_vp, _P(_i32), _P(_i32), _P(_i32), _P(_i32)],
    "rcs_circuit_one_qubit_gates": [_vp, _P(_i32)],
    "rcs_circuit_schedule": [_vp, _P(_i32), _P(_i32)],
    "rcs_build_state": [_vp, _i32, _d, _P(_vp)],
    "rcs_build_state_ex": [_vp, _i32, _d, _P(BuildOpts), _P(_vp)],
    "rcs_build_batch": [_P(_vp), _P(_i32), _P(_d), _i32, _P(BuildOpts), _P(_vp)],
    "rcs_sample": [_vp, _u64, _u64, _vp, _vp],
    "rcs_sample_range": [_vp, _u64, _u64, _u64, _vp, _vp],
    "rcs_sample_range_noalloc": [_vp, _u64, _u64, _u64, _vp, _vp],
    "rcs_sample_batch": [_P(_vp), _i32, _u64, _u64, _vp, _vp],
    "rcs_amplitudes": [_vp, _vp, _u64, _vp],
    "rcs_xeb": [_i32, _vp, _u64, _P(_d), _P(_d)],
    "rcs_xeb_log2": [_i32, _vp, _u64, _P(_d), _P(_d)],
    "rcs_xeb_state": [_vp, _vp, _u64, _P(_d), _P(_d)],
    "rcs_state_info_get": [_vp, _P(StateInfo)],
    "rcs_state_layout": [_vp, _P(_i32), _P(_i32)],
    "rcs_state_set_stream": [_vp, _vp],
    "rcs_state_export": [_vp, _P(_d), _i64, _P(_i64)],
    "rcs_state_import": [_i32, _P(_i32), _P(_i32), _P(_d), _i32, _vp, _P(_vp)],
    "rcs_state_save": [_vp, C.c_char_p],
    "rcs_state_load": [C.c_char_p, _vp, _P(_vp)],
    "rcs_state_spectra": [_vp, _P(_i32), _P(_i64), _P(_i32), _P(_d)],
    "rcs_state_updates": [_vp, _P(_i32), _P(_i32)],
    "rcs_state_rsvd_log": [_vp, _P(_i32), _P(_i64), _P(_i32), _P(_d), _P(C.c_float), _P(_d)],
    "rcs_svd_jacobi": [_i32, _i32, _vp, _vp, _vp, _vp],
    "rcs_svd_jacobi_f32": [_i32, _i32, _vp, _vp, _vp, _vp],
    "rcs_dense_simulate": [_vp, _vp, _i64, _vp],
    "rcs_dense_gather": [_vp, _i32, _vp, _u64, _i32, _vp, _vp],
    "rcs_cholqr": [_i32, _i32, _vp, _vp, _vp, _vp],
    "rcs_two_site": [_i32, _i32, _i32, _vp, _vp, _P(_d), _i32, _vp, _vp],
    "rcs_rsvd": [_i32, _i32, _vp, _i32, _i32, _u64, _u64, _vp, _P(_d), _vp],
    "rcs_rsvd_basis": [_i32, _i32, _vp, _i32, _i32, _u64, _u64, _vp, _vp],
    "rcs_spectrum_features": [_vp, _i32, _i32, _i32, _i32, _i32, _vp, _vp],
    "rcs_spectrum_targets": [_vp, _i32, _vp, _vp],
    "rcs_mlp_forward": [_vp, _vp, _i32, _vp, _vp],
    "rcs_mlp_backward": [_vp, _vp, _vp, _i32, _vp, _vp, _vp],
    "rcs_profile_enable": [_i32],
    "rcs_profile_event_floor": [_P(_d)],
    "rcs_tuning_set": [_i32, _i32, _i32],
    "rcs_profile_read": [_i32, _P(_i64), _P(_i64), _P(_d), _P(_d), _P(_d)],
    "rcs_mlp_adam": [_vp, _vp, _vp, _vp, _i32, _i32, C.c_float, C.c_float, C.c_float,
                     C.c_float, _vp],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.rcs_last_error.restype = C.c_char_p
_lib.rcs_version.restype = C.c_char_p
_lib.rcs_tuning_clear.argtypes = []
_lib.rcs_tuning_clear.restype = None
_lib.rcs_profile_class_name.argtypes = [_i32]
_lib.rcs_profile_class_name.restype = C.c_char_p
_lib.rcs_circuit_destroy.argtypes = [_vp]
_lib.rcs_circuit_destroy.restype = None
_lib.rcs_state_destroy.argtypes = [_vp]
_lib.rcs_state_destroy.restype = None
_lib.rcs_build_opts_default.argtypes = [_P(BuildOpts)]
_lib.rcs_build_opts_default.restype = None

EXPORTED = sorted(list(_SIGS) + ["rcs_last_error", "rcs_version", "rcs_circuit_destroy",
                                 "rcs_state_destroy", "rcs_build_opts_default",
                                 "rcs_profile_class_name", "rcs_tuning_clear"])
KERNEL_CLASSES = ["k_chain_gemm", "k_jac_gram", "k_jac_rotate", "k_two_site", "k_range_finder",
                  "k_factor_other"]


def _check(st):
    if st != 0:
        raise RcsError(st, _lib.rcs_last_error().decode())


def version():
    return _lib.rcs_version().decode()


def _ptr(t):
    """Device (or host) pointer of a contiguous torch tensor."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    if stream is None:
        return None
    return C.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ circuits
class Circuit:
    def __init__(self, rows, cols, n_cycles, seed, pattern="ABCDCDAB", removed=(),
                 n_removed_random=0, theta=np.pi / 2, phi=np.pi / 6, final_1q_layer=True,
                 network="snake", lattice="rect"):
        rem = (C.c_int32 * max(1, len(removed)))(*removed)
        self._pattern = pattern.encode() if pattern is not None else None
        self.network = network
        d = CircuitDesc(rows, cols, n_cycles, seed & 0xFFFFFFFFFFFFFFFF, len(removed),
                        C.cast(rem, _P(C.c_int32)), n_removed_random, self._pattern,
                        float(theta), float(phi), 1 if final_1q_layer else 0, NETWORKS[network],
                        LATTICES[lattice])
        h = C.c_void_p()
        _check(_lib.rcs_circuit_create(C.byref(d), C.byref(h)))
        self.h = h
        n, nl, no, nu = _i32(), _i32(), _i32(), _i32()
        _check(_lib.rcs_circuit_info(h, C.byref(n), C.byref(nl), C.byref(no), C.byref(nu)))
        self.n, self.n_layers_1q, self.n_ops, self.n_updates = n.value, nl.value, no.value, nu.value

    def one_qubit_gates(self):
        out = np.zeros(self.n_layers_1q * self.n, dtype=np.int32)
        _check(_lib.rcs_circuit_one_qubit_gates(self.h, out.ctypes.data_as(_P(_i32))))
        return out.reshape(self.n_layers_1q, self.n)

    def schedule(self):
        snake = np.zeros(self.n, dtype=np.int32)
        ops = np.zeros(4 * self.n_ops, dtype=np.int32)
        _check(_lib.rcs_circuit_schedule(self.h, snake.ctypes.data_as(_P(_i32)),
                                         ops.ctypes.data_as(_P(_i32))))
        return snake, ops.reshape(self.n_ops, 4)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.rcs_circuit_destroy(h)
            self.h = None


# ------------------------------------------------------------------- states
def build_opts(contraction="c128", rank_mode=RCS_RANK_FULL_SVD, fallback_tau=1e-6,
               mlp_weights=None, rsvd_oversample=16, rsvd_power_iters=2, rsvd_seed=0x5EED,
               stream=None, log_spectra=False, max_ops=-1, canonicalize=True, svd_precision="f64"):
    o = BuildOpts()
    _lib.rcs_build_opts_default(C.byref(o))
    o.contraction = PRECISIONS[contraction] if isinstance(contraction, str) else int(contraction)
    o.rank_mode = int(rank_mode)
    o.fallback_tau = float(fallback_tau)
    keep = None
    if mlp_weights is not None:
        keep = np.ascontiguousarray(mlp_weights, dtype=np.float32)
        o.mlp_weights_host = keep.ctypes.data_as(_P(C.c_float))
        o.mlp_count = keep.size
    o.rsvd_oversample = rsvd_oversample
    o.rsvd_power_iters = rsvd_power_iters
    o.rsvd_seed = rsvd_seed
    o.stream = _stream_ptr(stream)
    o.log_spectra = 1 if log_spectra else 0
    o.max_ops = max_ops
    o.canonicalize = 1 if canonicalize else 0
    o.svd_precision = SVD_PRECISIONS[svd_precision] if isinstance(svd_precision, str) else int(svd_precision)
    return o, keep


class State:
    def __init__(self, handle):
        self.h = handle
        self.n = self.info().n_qubits

    @staticmethod
    def build(circuit, chi, eps, **kw):
        o, keep = build_opts(**kw)
        h = C.c_void_p()
        _check(_lib.rcs_build_state_ex(circuit.h, int(chi), float(eps), C.byref(o), C.byref(h)))
        del keep
        return State(h)

    @staticmethod
    def build_batch(circuits, chis, epss, **kw):
        o, keep = build_opts(**kw)
        n = len(circuits)
        hs = (C.c_void_p * n)(*[c.h for c in circuits])
        ch = (C.c_int32 * n)(*chis)
        ep = (C.c_double * n)(*epss)
        out = (C.c_void_p * n)()
        _check(_lib.rcs_build_batch(hs, ch, ep, n, C.byref(o), out))
        del keep
        return [State(C.c_void_p(out[i])) for i in range(n)]

    @staticmethod
    def from_host(dims, snake, tensors, canonical=True, stream=None):
        """tensors: list of complex128 arrays A_k (dims[k], 2, dims[k+1])."""
        dims = np.ascontiguousarray(dims, dtype=np.int32)
        snake = np.ascontiguousarray(snake, dtype=np.int32)
        flat = np.concatenate([np.ascontiguousarray(a, dtype=np.complex128).reshape(-1)
                               for a in tensors]).view(np.float64)
        h = C.c_void_p()
        _check(_lib.rcs_state_import(len(snake), dims.ctypes.data_as(_P(_i32)),
                                     snake.ctypes.data_as(_P(_i32)),
                                     flat.ctypes.data_as(_P(_d)), 1 if canonical else 0,
                                     _stream_ptr(stream), C.byref(h)))
        return State(h)

    @staticmethod
    def load(path, stream=None):
        """A state saved by State.save (rcs_state_load)."""
        h = C.c_void_p()
        _check(_lib.rcs_state_load(os.fsencode(path), _stream_ptr(stream), C.byref(h)))
        return State(h)

    def save(self, path):
        """Persist the state (rcs_state_save)."""
        _check(_lib.rcs_state_save(self.h, os.fsencode(path)))

    def info(self):
        inf = StateInfo()
        _check(_lib.rcs_state_info_get(self.h, C.byref(inf)))
        return inf

    def layout(self):
        n = self.n
        dims = np.zeros(max(n - 1, 1), dtype=np.int32)
        snake = np.zeros(n, dtype=np.int32)
        _check(_lib.rcs_state_layout(self.h, dims.ctypes.data_as(_P(_i32)),
                                     snake.ctypes.data_as(_P(_i32))))
        return dims[:n - 1], snake

    def set_stream(self, stream):
        _check(_lib.rcs_state_set_stream(self.h, _stream_ptr(stream)))

    def to_host(self):
        need = _i64()
        _check(_lib.rcs_state_export(self.h, None, 0, C.byref(need)))
        buf = np.zeros(need.value, dtype=np.float64)
        _check(_lib.rcs_state_export(self.h, buf.ctypes.data_as(_P(_d)), need.value, None))
        bonds, snake = self.layout()
        dims = [1] + list(bonds) + [1]
        z = buf.view(np.complex128)
        out, o = [], 0
        for k in range(self.n):
            sz = dims[k] * 2 * dims[k + 1]
            out.append(z[o:o + sz].reshape(dims[k], 2, dims[k + 1]).copy())
            o += sz
        return dims, snake, out

    def spectra(self):
        nr, nv = _i32(), _i64()
        _check(_lib.rcs_state_spectra(self.h, C.byref(nr), C.byref(nv), None, None))
        meta = np.zeros(6 * max(nr.value, 1), dtype=np.int32)
        vals = np.zeros(max(nv.value, 1), dtype=np.float64)
        _check(_lib.rcs_state_spectra(self.h, C.byref(nr), C.byref(nv),
                                      meta.ctypes.data_as(_P(_i32)), vals.ctypes.data_as(_P(_d))))
        meta = meta[:6 * nr.value].reshape(nr.value, 6)
        out, o = [], 0
        for r in meta:
            m = int(r[2])
            out.append(dict(pos=int(r[0]), cycle=int(r[1]), m=m, kept=int(r[3]),
                            chi_l=int(r[4]), chi_r=int(r[5]), values=vals[o:o + m].copy()))
            o += m
        return out

    def updates(self):
        """(n_updates, 7) int32: position, cycle, chi_l, chi_m, chi_r, kept,
        path (0 full SVD, 1 randomized accepted, 2 randomized rejected)."""
        n = _i32()
        _check(_lib.rcs_state_updates(self.h, C.byref(n), None))
        rec = np.zeros(7 * max(n.value, 1), dtype=np.int32)
        _check(_lib.rcs_state_updates(self.h, C.byref(n), rec.ctypes.data_as(_P(_i32))))
        return rec[:7 * n.value].reshape(n.value, 7)

    def rsvd_log(self):
        """One dict per randomized split: the decisions of the learned path."""
        nr, nv = _i32(), _i64()
        _check(_lib.rcs_state_rsvd_log(self.h, C.byref(nr), C.byref(nv), None, None, None, None))
        n = nr.value
        ints = np.zeros(10 * max(n, 1), dtype=np.int32)
        dbl = np.zeros(4 * max(n, 1), dtype=np.float64)
        net = np.zeros(98 * max(n, 1), dtype=np.float32)
        vals = np.zeros(max(nv.value, 1), dtype=np.float64)
        _check(_lib.rcs_state_rsvd_log(self.h, C.byref(nr), C.byref(nv),
                                       ints.ctypes.data_as(_P(_i32)), dbl.ctypes.data_as(_P(_d)),
                                       net.ctypes.data_as(_P(C.c_float)),
                                       vals.ctypes.data_as(_P(_d))))
        out, o = [], 0
        for r in range(n):
            q = ints[10 * r:10 * r + 10]
            d = dbl[4 * r:4 * r + 4]
            nvr = int(q[9])
            out.append(dict(update=int(q[0]), pos=int(q[1]), cycle=int(q[2]), m=int(q[3]),
                            k_hat=int(q[4]), l=int(q[5]), k=int(q[6]), accepted=bool(q[7]),
                            early=bool(q[8]), eps_pred=float(d[0]), eps_rand=float(d[1]),
                            outside=float(d[2]), total=float(d[3]),
                            feat=net[98 * r:98 * r + 66].copy(), y=net[98 * r + 66:98 * r + 98].copy(),
                            values=vals[o:o + nvr].copy()))
            o += nvr
        return out

    def sample(self, bits, log2p=None, n_shots=None, seed=0, first_shot=0):
        """bits: uint64/int64 device tensor (n_shots,); log2p: float64 or None."""
        n_shots = bits.numel() if n_shots is None else n_shots
        _check(_lib.rcs_sample_range(self.h, first_shot, n_shots, seed & 0xFFFFFFFFFFFFFFFF,
                                     _ptr(bits), _ptr(log2p)))

    def sample_noalloc(self, bits, log2p=None, n_shots=None, seed=0, first_shot=0):
        """As sample(), through the allocation-free entry point (the library's
        static per-device scratch array instead of allocated workspace)."""
        n_shots = bits.numel() if n_shots is None else n_shots
        _check(_lib.rcs_sample_range_noalloc(self.h, first_shot, n_shots, seed & 0xFFFFFFFFFFFFFFFF,
                                             _ptr(bits), _ptr(log2p)))

    def amplitudes(self, bits, amps):
        """amps: float64 device tensor (m, 2) or complex128 (m,)."""
        _check(_lib.rcs_amplitudes(self.h, _ptr(bits), bits.numel(), _ptr(amps)))

    def xeb_of(self, bits):
        x, se = _d(), _d()
        _check(_lib.rcs_xeb_state(self.h, _ptr(bits), bits.numel(), C.byref(x), C.byref(se)))
        return x.value, se.value

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.rcs_state_destroy(h)
            self.h = None


def sample_batch(states, n_shots, seed, bits, log2p=None):
    n = len(states)
    hs = (C.c_void_p * n)(*[s.h for s in states])
    _check(_lib.rcs_sample_batch(hs, n, n_shots, seed, _ptr(bits), _ptr(log2p)))


def xeb(n_qubits, p_ref):
    x, se = _d(), _d()
    _check(_lib.rcs_xeb(n_qubits, _ptr(p_ref), p_ref.numel(), C.byref(x), C.byref(se)))
    return x.value, se.value


def xeb_log2(n_qubits, log2p):
    x, se = _d(), _d()
    _check(_lib.rcs_xeb_log2(n_qubits, _ptr(log2p), log2p.numel(), C.byref(x), C.byref(se)))
    return x.value, se.value


# ------------------------------------------------------------ kernel-level
def svd_jacobi(x, s, u, stream=None):
    """x: complex128 device tensor (cnt, len) holding the columns (column-major
    len x cnt matrix); overwritten.  s: float64 (cnt,), u: complex128 like x."""
    cnt, ln = x.shape
    _check(_lib.rcs_svd_jacobi(ln, cnt, _ptr(x), _ptr(s), _ptr(u), _stream_ptr(stream)))


def svd_jacobi_f32(x, s, u, stream=None):
    """As svd_jacobi with the Jacobi in fp32; x (complex128) is not modified."""
    cnt, ln = x.shape
    _check(_lib.rcs_svd_jacobi_f32(ln, cnt, _ptr(x), _ptr(s), _ptr(u), _stream_ptr(stream)))


def dense_simulate(circuit, psi, stream=None):
    """psi: complex128 device tensor of 2^n entries, overwritten with the
    circuit's exact output state (index bit q = qubit q)."""
    _check(_lib.rcs_dense_simulate(circuit.h, _ptr(psi), psi.numel(), _stream_ptr(stream)))


def dense_gather(psi, n_qubits, bits, out, probabilities=True, stream=None):
    """out[i] = |psi[bits[i]]|^2 (float64) or psi[bits[i]] (complex128)."""
    _check(_lib.rcs_dense_gather(_ptr(psi), n_qubits, _ptr(bits), bits.numel(), 1 if probabilities else 0,
                                 _ptr(out), _stream_ptr(stream)))


def cholqr(x, q, r, stream=None):
    """x: complex128 device tensor (cnt, len) holding the columns of a
    column-major len x cnt matrix (not modified); q: like x; r: complex128
    (cnt, cnt) receiving the columns of R (X = Q R, Q orthonormal)."""
    cnt, ln = x.shape
    _check(_lib.rcs_cholqr(ln, cnt, _ptr(x), _ptr(q), _ptr(r), _stream_ptr(stream)))


def two_site(a, b, gate, out, precision="c128", stream=None):
    """a: (dl,2,dm), b: (dm,2,dr) complex128 device tensors; out: complex128
    (2dr, 2dl) holding the (2dl)x(2dr) matrix column-major."""
    dl, _, dm = a.shape
    dr = b.shape[2]
    g = np.ascontiguousarray(gate, dtype=np.complex128).reshape(-1).view(np.float64)
    _check(_lib.rcs_two_site(dl, dm, dr, _ptr(a), _ptr(b), g.ctypes.data_as(_P(_d)),
                             PRECISIONS[precision], _ptr(out), _stream_ptr(stream)))


def rsvd(x, l, q, seed, step, s, stream=None):
    cnt, ln = x.shape
    f = _d()
    _check(_lib.rcs_rsvd(ln, cnt, _ptr(x), l, q, seed, step, _ptr(s), C.byref(f),
                         _stream_ptr(stream)))
    return f.value


def rsvd_basis(x, l, q, seed, step, qout, stream=None):
    """qout: complex128 device tensor (l, len) receiving the basis columns."""
    cnt, ln = x.shape
    _check(_lib.rcs_rsvd_basis(ln, cnt, _ptr(x), l, q, seed, step, _ptr(qout), _stream_ptr(stream)))


def spectrum_features(s, k, bond, n_sites, cycle, n_cycles, feat, stream=None):
    _check(_lib.rcs_spectrum_features(_ptr(s), k, bond, n_sites, cycle, n_cycles, _ptr(feat),
                                      _stream_ptr(stream)))


def spectrum_targets(s, m, y, stream=None):
    _check(_lib.rcs_spectrum_targets(_ptr(s), m, _ptr(y), _stream_ptr(stream)))


def mlp_forward(w, x, out, stream=None):
    _check(_lib.rcs_mlp_forward(_ptr(w), _ptr(x), x.shape[0], _ptr(out), _stream_ptr(stream)))


def mlp_backward(w, x, y, grad, loss, stream=None):
    _check(_lib.rcs_mlp_backward(_ptr(w), _ptr(x), _ptr(y), x.shape[0], _ptr(grad), _ptr(loss),
                                 _stream_ptr(stream)))


def mlp_adam(w, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(_lib.rcs_mlp_adam(_ptr(w), _ptr(grad), _ptr(m), _ptr(v), w.numel(), step, lr, beta1,
                             beta2, eps, _stream_ptr(stream)))


# ------------------------------------------------------------- measurement
def profile_enable(every):
    _check(_lib.rcs_profile_enable(int(every)))


def profile_event_floor():
    """Seconds of an empty kernel timed like a probed launch."""
    v = _d()
    _check(_lib.rcs_profile_event_floor(C.byref(v)))
    return v.value


def profile_read(kclass):
    """dict(launches, timed, seconds, flops, bytes) of one kernel class."""
    a, b = _i64(), _i64()
    sec, fl, by = _d(), _d(), _d()
    _check(_lib.rcs_profile_read(int(kclass), C.byref(a), C.byref(b), C.byref(sec), C.byref(fl),
                                 C.byref(by)))
    return dict(name=_lib.rcs_profile_class_name(int(kclass)).decode(), launches=a.value,
                timed=b.value, seconds=sec.value, flops=fl.value, bytes=by.value)


def tuning_set(cnt_max, block, inner_sweeps):
    _check(_lib.rcs_tuning_set(int(cnt_max), int(block), int(inner_sweeps)))


def tuning_clear():
    _lib.rcs_tuning_clear()
