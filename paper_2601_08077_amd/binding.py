"""ctypes binding of libdfjk.so: the C ABI of include/dfjk.h, same names.

Argument marshalling only: torch tensors provide device pointers and the HIP
stream; every step of the build runs in the library's kernels.  Importing
works without a GPU; loading the library fails loudly if it was not built.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdfjk.so")

DF_OK, DF_EINVAL, DF_EWORKSPACE, DF_EHIP, DF_ENONFINITE, DF_EOVERFLOW_GUARD, DF_ENOTSPD = (
    0, -1, -2, -3, -4, -5, -6)
DF_DENSE, DF_PACKED = 0, 1
STAGES = ("bexp", "prep", "x", "slice_x", "k", "k_reduce", "rho", "j", "energies", "bound")

_c_void_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int


class DFProblem(ctypes.Structure):
    """struct df_problem of dfjk.h (one instance of the batched build)."""
    _fields_ = [("B", _c_void_p), ("b_exp", _c_void_p), ("naux", _i64), ("nao", _i64),
                ("nocc", _i64), ("C", _c_void_p), ("D", _c_void_p), ("occ", ctypes.c_double),
                ("slices", _int), ("screen_mask", _c_void_p), ("screen_chunks", _c_void_p),
                ("screen_blk", _int), ("J", _c_void_p), ("K", _c_void_p),
                ("energies", _c_void_p), ("err_bound", _c_void_p)]

# name -> (restype, argtypes)
SIGNATURES = {
    "df_create": (_int, [ctypes.POINTER(_c_void_p), _c_void_p]),
    "df_destroy": (None, [_c_void_p]),
    "df_set_precision": (_int, [_c_void_p, _int]),
    "df_get_precision": (_int, [_c_void_p]),
    "df_set_pblk": (_int, [_c_void_p, _int]),
    "df_set_k_groups": (_int, [_c_void_p, _int]),
    "df_set_block_precision": (_int, [_c_void_p, ctypes.POINTER(ctypes.c_int32), _i64]),
    "df_get_k_groups": (_int, [_c_void_p]),
    "df_set_x_ksub": (_int, [_c_void_p, _int]),
    "df_set_extra_pairs": (_int, [_c_void_p, _int]),
    "df_workspace_size": (_int, [_c_void_p, _i64, _i64, _i64, _int, ctypes.POINTER(ctypes.c_size_t)]),
    "df_set_workspace": (_int, [_c_void_p, _c_void_p, ctypes.c_size_t]),
    "df_b_exponents": (_int, [_c_void_p, _c_void_p, _int, _i64, _i64, _c_void_p]),
    "df_slice": (_int, [_c_void_p, _c_void_p, _i64, _i64, _i64, _int, _c_void_p, _c_void_p]),
    "df_build_x": (_int, [_c_void_p, _c_void_p, _int, _i64, _i64, _c_void_p, _c_void_p, _i64,
                          _c_void_p]),
    "df_build_jk": (_int, [_c_void_p, _c_void_p, _int, _i64, _i64, _c_void_p, _c_void_p, _i64,
                           ctypes.c_double, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p]),
    "df_build_jk_noalloc": (_int, [_c_void_p, _c_void_p, _int, _i64, _i64, _c_void_p, _c_void_p,
                                   _i64, ctypes.c_double, _c_void_p, _c_void_p, _c_void_p,
                                   _c_void_p, _c_void_p]),
    "df_prepare_b_size": (_int, [_i64, _i64, _int, ctypes.POINTER(ctypes.c_size_t)]),
    "df_prepare_b": (_int, [_c_void_p, _c_void_p, _int, _i64, _i64, _int, _c_void_p, _c_void_p]),
    "df_build_jk_sliced": (_int, [_c_void_p, _c_void_p, _int, _c_void_p, _i64, _i64, _c_void_p,
                                  _i64, ctypes.c_double, _c_void_p, _c_void_p, _c_void_p,
                                  _c_void_p, _c_void_p]),
    "df_block_stats": (_int, [_c_void_p, _c_void_p, _c_void_p, _i64, _i64, _c_void_p]),
    "df_x_block_stats": (_int, [_c_void_p, _i64, _i64, _i64, _c_void_p]),
    "df_controller_features": (_int, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                                      _c_void_p, ctypes.POINTER(ctypes.c_double), _i64,
                                      _c_void_p]),
    "df_mlp_nparams": (_int, []),
    "df_mlp_forward": (_int, [_c_void_p, _c_void_p, _c_void_p, _i64, _c_void_p]),
    "df_mlp_train_step": (_int, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _i64, _c_void_p,
                                 _c_void_p, _c_void_p, _c_void_p, _i64, ctypes.c_float,
                                 _c_void_p]),
    "df_choose_slices": (_int, [_c_void_p, _c_void_p, _i64, ctypes.c_double, _c_void_p]),
    "df_block_partials": (_int, [_c_void_p, _i64, _i64, _i64, _c_void_p]),
    "df_block_errors": (_int, [_c_void_p, _i64, _i64, _i64, ctypes.c_double, _c_void_p,
                               ctypes.c_double, _c_void_p]),
    "df_spot_check": (_int, [_c_void_p, _c_void_p, _int, _i64, _i64, _c_void_p, _i64,
                             ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                             _int, _c_void_p]),
    "df_controller_allocate": (_int, [ctypes.POINTER(ctypes.c_float), _i64, _int, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int32)]),
    "df_screen": (_int, [_c_void_p, _c_void_p, _i64, _i64, _int, ctypes.c_double, _c_void_p,
                         _c_void_p, _c_void_p]),
    "df_set_screening": (_int, [_c_void_p, _c_void_p, _c_void_p, _int, _i64]),
    "df_autotune": (_int, [_c_void_p, _c_void_p, _c_void_p, _i64, _i64, _c_void_p, _i64,
                           ctypes.c_double, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                           _int, ctypes.POINTER(_int), ctypes.POINTER(_int),
                           ctypes.POINTER(ctypes.c_double)]),
    "df_batched_workspace_size": (_int, [_c_void_p, _int, ctypes.POINTER(DFProblem), _int,
                                         ctypes.POINTER(ctypes.c_size_t)]),
    "df_build_jk_batched": (_int, [_c_void_p, _int, ctypes.POINTER(DFProblem), _int]),
    "df_get_status": (_int, [_c_void_p]),
    "df_last_error": (ctypes.c_char_p, [_c_void_p]),
    "df_metric_cholesky": (_int, [_c_void_p, _c_void_p, _i64]),
    "df_whiten": (_int, [_c_void_p, _c_void_p, _i64, _c_void_p, _i64, _c_void_p]),
    "df_density": (_int, [_c_void_p, _c_void_p, _i64, _i64, ctypes.c_double, _c_void_p]),
    "df_fock": (_int, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _i64, _c_void_p,
                       _c_void_p]),
    "df_rule_level": (_int, [ctypes.c_double]),
    "df_rule_next_level": (_int, [_int, ctypes.c_double, ctypes.c_double]),
    "df_rule_slices": (_int, [_int, _int]),
    "df_peak_probe": (_int, [_c_void_p, _int, _c_void_p, ctypes.c_size_t, _int,
                             ctypes.POINTER(ctypes.c_double)]),
    "df_timing_begin": (_int, [_c_void_p, _int]),
    "df_timing_end": (_int, [_c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_int)]),
    "df_debug_build_i32": (_int, [_c_void_p, _c_void_p, _int, _i64, _i64, _c_void_p, _c_void_p,
                                  _i64, _c_void_p, _c_void_p]),
    "df_debug_slice_gemm_i32": (_int, [_c_void_p, _c_void_p, _c_void_p, _i64, _i64, _i64, _int,
                                       _c_void_p]),
}

_lib = None


def load():
    """Load libdfjk.so (once) and declare every exported signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2601_08077_amd.build` (hipcc, gfx950)")
    # torch's HIP runtime must be the one in the process before the library
    # binds to libamdhip64 (both carry the same soname): import it first.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class DFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _shape(B, layout, naux=None, nao=None):
    """(naux, nao) of B: [naux][nao][nao] (DF_DENSE) or [naux][nao (nao + 1) / 2]
    (DF_PACKED; nao follows from the packed length unless given)."""
    if naux is None:
        naux = B.shape[0]
    if nao is None:
        if layout == DF_PACKED:
            import math
            npair = B.shape[1]
            nao = (math.isqrt(8 * npair + 1) - 1) // 2
            if nao * (nao + 1) // 2 != npair:
                raise ValueError("packed B: the row length is not a triangular number")
        else:
            nao = B.shape[1]
    return int(naux), int(nao)


class Context:
    """A df_ctx bound to a torch CUDA(HIP) stream, plus its workspace tensor."""

    def __init__(self, stream=None):
        import torch
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.df_create(ctypes.byref(h), ctypes.c_void_p(stream.cuda_stream))
        if rc != DF_OK:
            raise DFError(rc, "df_create failed")
        self.h = h
        self.ws = None

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.df_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != DF_OK:
            msg = self.lib.df_last_error(self.h)
            raise DFError(rc, f"{what}: {msg.decode() if msg else ''}")

    # -- configuration --------------------------------------------------------
    def df_set_precision(self, slices):
        self._check(self.lib.df_set_precision(self.h, int(slices)), "df_set_precision")

    def df_get_precision(self):
        return self.lib.df_get_precision(self.h)

    def df_set_pblk(self, pblk):
        self._check(self.lib.df_set_pblk(self.h, int(pblk)), "df_set_pblk")

    def df_set_k_groups(self, groups):
        self._check(self.lib.df_set_k_groups(self.h, int(groups)), "df_set_k_groups")

    def df_set_block_precision(self, s_blocks):
        """Per-aux-block slice counts (sequence of ints 0..8), or None to reset."""
        if s_blocks is None:
            self._check(self.lib.df_set_block_precision(self.h, None, 0), "df_set_block_precision")
            return
        arr = (ctypes.c_int32 * len(s_blocks))(*[int(v) for v in s_blocks])
        self._check(self.lib.df_set_block_precision(self.h, arr, len(s_blocks)),
                    "df_set_block_precision")

    def df_set_extra_pairs(self, extra):
        self._check(self.lib.df_set_extra_pairs(self.h, int(extra)), "df_set_extra_pairs")

    def df_set_x_ksub(self, ksub):
        self._check(self.lib.df_set_x_ksub(self.h, int(ksub)), "df_set_x_ksub")

    def df_get_k_groups(self):
        return self.lib.df_get_k_groups(self.h)

    def df_workspace_size(self, naux, nao, nocc, layout=DF_DENSE):
        n = ctypes.c_size_t()
        self._check(self.lib.df_workspace_size(self.h, naux, nao, nocc, layout, ctypes.byref(n)),
                    "df_workspace_size")
        return n.value

    def df_set_workspace(self, ws):
        """Hand over a uint8 device tensor (kept alive by this object)."""
        self.ws = ws
        self._check(self.lib.df_set_workspace(self.h, _ptr(ws), 0 if ws is None else ws.numel()),
                    "df_set_workspace")

    def ensure_workspace(self, naux, nao, nocc, layout=DF_DENSE):
        import torch
        need = self.df_workspace_size(naux, nao, nocc, layout)
        if self.ws is None or self.ws.numel() < need:
            self.df_set_workspace(None)
            self.df_set_workspace(torch.empty(need, dtype=torch.uint8, device="cuda"))
        return need

    # -- compute entry points -------------------------------------------------
    def df_b_exponents(self, B, b_exp, layout=DF_DENSE, naux=None, nao=None):
        naux, nao = _shape(B, layout, naux, nao)
        self._check(self.lib.df_b_exponents(self.h, _ptr(B), layout, naux, nao, _ptr(b_exp)),
                    "df_b_exponents")

    def df_slice(self, A, slices, digits, row_exp):
        rows, cols = A.shape
        self._check(self.lib.df_slice(self.h, _ptr(A), rows, cols, A.stride(0), int(slices),
                                      _ptr(digits), _ptr(row_exp)), "df_slice")

    def df_build_x(self, B, b_exp, C, X, layout=DF_DENSE, naux=None, nao=None):
        naux, nao = _shape(B, layout, naux, nao)
        self._check(self.lib.df_build_x(self.h, _ptr(B), layout, naux, nao, _ptr(b_exp), _ptr(C),
                                        C.shape[1], _ptr(X)), "df_build_x")

    def df_build_jk(self, B, b_exp, C, occ, D, J, K, energies, err_bound, layout=DF_DENSE,
                    naux=None, nao=None):
        naux, nao = _shape(B, layout, naux, nao)
        self._check(self.lib.df_build_jk(self.h, _ptr(B), layout, naux, nao, _ptr(b_exp), _ptr(C),
                                         C.shape[1], float(occ), _ptr(D), _ptr(J), _ptr(K),
                                         _ptr(energies), _ptr(err_bound)), "df_build_jk")

    def df_build_jk_noalloc(self, B, b_exp, C, occ, D, J, K, energies, err_bound,
                            layout=DF_DENSE, naux=None, nao=None):
        """df_build_jk on the library's static 64 MiB workspace (no allocation)."""
        naux, nao = _shape(B, layout, naux, nao)
        self._check(self.lib.df_build_jk_noalloc(self.h, _ptr(B), layout, naux, nao, _ptr(b_exp),
                                                 _ptr(C), C.shape[1], float(occ), _ptr(D),
                                                 _ptr(J), _ptr(K), _ptr(energies),
                                                 _ptr(err_bound)), "df_build_jk_noalloc")

    def df_prepare_b(self, B, planes, b_exp, b_dig, layout=DF_DENSE, naux=None, nao=None):
        """b_exp [naux*nao] int32, b_dig [planes][naux*nao][ldk] int8 (ldk = nao
        rounded up to 64); sizes from df_prepare_b_size."""
        naux, nao = _shape(B, layout, naux, nao)
        self._check(self.lib.df_prepare_b(self.h, _ptr(B), layout, naux, nao, int(planes),
                                          _ptr(b_exp), _ptr(b_dig)), "df_prepare_b")

    def df_build_jk_sliced(self, b_dig, planes, b_exp, naux, nao, C, occ, D, J, K, energies,
                           err_bound):
        """err_bound: 2 doubles (K bound, J bound)."""
        self._check(self.lib.df_build_jk_sliced(self.h, _ptr(b_dig), int(planes), _ptr(b_exp),
                                                naux, nao, _ptr(C), C.shape[1], float(occ),
                                                _ptr(D), _ptr(J), _ptr(K), _ptr(energies),
                                                _ptr(err_bound)), "df_build_jk_sliced")

    # -- learned slice controller -------------------------------------------------
    def df_block_stats(self, A, out, seglen, A2=None):
        self._check(self.lib.df_block_stats(self.h, _ptr(A), _ptr(A2), A.numel(), int(seglen),
                                            _ptr(out)), "df_block_stats")

    def df_x_block_stats(self, naux, nao, nocc, out):
        self._check(self.lib.df_x_block_stats(self.h, naux, nao, nocc, _ptr(out)),
                    "df_x_block_stats")

    def df_controller_features(self, bstats, xstats, dstat, cstat, kstat, scalars, feat):
        sc = (ctypes.c_double * 8)(*[float(v) for v in scalars])
        self._check(self.lib.df_controller_features(self.h, _ptr(bstats), _ptr(xstats),
                                                    _ptr(dstat), _ptr(cstat), _ptr(kstat), sc,
                                                    feat.shape[0], _ptr(feat)),
                    "df_controller_features")

    def df_mlp_forward(self, params, x, y):
        self._check(self.lib.df_mlp_forward(self.h, _ptr(params), _ptr(x), x.shape[0], _ptr(y)),
                    "df_mlp_forward")

    def df_mlp_train_step(self, params, m, v, step, x, t, mask, idx, n, lr, loss=None):
        self._check(self.lib.df_mlp_train_step(self.h, _ptr(params), _ptr(m), _ptr(v), int(step),
                                               _ptr(x), _ptr(t), _ptr(mask), _ptr(idx), int(n),
                                               float(lr), _ptr(loss)), "df_mlp_train_step")

    def df_choose_slices(self, pred, target, s_out):
        self._check(self.lib.df_choose_slices(self.h, _ptr(pred), pred.shape[0], float(target),
                                              _ptr(s_out)), "df_choose_slices")

    def df_block_partials(self, naux, nao, nocc, out):
        self._check(self.lib.df_block_partials(self.h, naux, nao, nocc, _ptr(out)),
                    "df_block_partials")

    def df_block_errors(self, naux, nao, nocc, occ, kref, kfro, err):
        self._check(self.lib.df_block_errors(self.h, naux, nao, nocc, float(occ), _ptr(kref),
                                             float(kfro), _ptr(err)), "df_block_errors")

    def df_spot_check(self, B, C, occ, kfro, blocks, err, layout=DF_DENSE, naux=None, nao=None):
        naux, nao = _shape(B, layout, naux, nao)
        arr = (ctypes.c_int32 * len(blocks))(*[int(b) for b in blocks])
        self._check(self.lib.df_spot_check(self.h, _ptr(B), layout, naux, nao, _ptr(C),
                                           C.shape[1], float(occ), float(kfro), arr, len(blocks),
                                           _ptr(err)),
                    "df_spot_check")

    def df_screen(self, B, blk, tau, mask, chunks, norms=None):
        """Zeroes the dropped shell blocks of B in place; mask uint8 [nblk][nblk],
        chunks int64 [nao] (bit patterns), norms float64 [nblk][nblk] or None."""
        naux, nao = B.shape[0], B.shape[1]
        self._check(self.lib.df_screen(self.h, _ptr(B), naux, nao, int(blk), float(tau),
                                       _ptr(mask), _ptr(chunks), _ptr(norms)), "df_screen")

    def df_set_screening(self, mask, chunks, blk, nao):
        self._check(self.lib.df_set_screening(self.h, _ptr(mask), _ptr(chunks), int(blk), int(nao)),
                    "df_set_screening")

    def df_autotune(self, B, b_exp, C, occ, D, J, K, energies, err_bound, reps=3):
        """Returns (groups, ksub, ms) of the fastest launch shape, kept in the context."""
        naux, nao = B.shape[0], B.shape[1]
        g, k, ms = _int(), _int(), ctypes.c_double()
        self._check(self.lib.df_autotune(self.h, _ptr(B), _ptr(b_exp), naux, nao, _ptr(C),
                                         C.shape[1], float(occ), _ptr(D), _ptr(J), _ptr(K),
                                         _ptr(energies), _ptr(err_bound), int(reps),
                                         ctypes.byref(g), ctypes.byref(k), ctypes.byref(ms)),
                    "df_autotune")
        return g.value, k.value, ms.value

    @staticmethod
    def make_problem(B, C, D, J, K, energies, err_bound, slices, occ=2.0, b_exp=None,
                     screen_mask=None, screen_chunks=None, screen_blk=8):
        naux, nao = B.shape[0], B.shape[1]
        return DFProblem(B.data_ptr(), 0 if b_exp is None else b_exp.data_ptr(), naux, nao,
                         C.shape[1], C.data_ptr(), D.data_ptr(), float(occ), int(slices),
                         0 if screen_mask is None else screen_mask.data_ptr(),
                         0 if screen_chunks is None else screen_chunks.data_ptr(),
                         int(screen_blk), J.data_ptr(), K.data_ptr(), energies.data_ptr(),
                         err_bound.data_ptr())

    def df_batched_workspace_size(self, problems, streams):
        arr = (DFProblem * len(problems))(*problems)
        n = ctypes.c_size_t()
        self._check(self.lib.df_batched_workspace_size(self.h, len(problems), arr, int(streams),
                                                       ctypes.byref(n)),
                    "df_batched_workspace_size")
        return n.value

    def df_build_jk_batched(self, problems, streams):
        arr = (DFProblem * len(problems))(*problems)
        self._check(self.lib.df_build_jk_batched(self.h, len(problems), arr, int(streams)),
                    "df_build_jk_batched")

    def df_metric_cholesky(self, W):
        """In place: the lower triangle of W becomes L (L L^T = W), upper set to 0."""
        self._check(self.lib.df_metric_cholesky(self.h, _ptr(W), W.shape[0]), "df_metric_cholesky")

    def df_whiten(self, L, T, B):
        """B = L^-1 T (T, B: [naux][ncols]); the workspace must hold naux^2 doubles."""
        naux = L.shape[0]
        ncols = T.numel() // naux
        self._check(self.lib.df_whiten(self.h, _ptr(L), naux, _ptr(T), ncols, _ptr(B)), "df_whiten")

    def df_density(self, C, occ, D):
        self._check(self.lib.df_density(self.h, _ptr(C), C.shape[0], C.shape[1], float(occ), _ptr(D)),
                    "df_density")

    def df_peak_probe(self, kind, buf, iters=1):
        """Rate of peak probe `kind` (0 INT8 MFMA TOP/s, 1 FP64 MFMA TFLOP/s,
        2 copy GB/s, 3 read GB/s) on the uint8 device tensor buf."""
        r = ctypes.c_double()
        self._check(self.lib.df_peak_probe(self.h, int(kind), _ptr(buf), buf.numel(), int(iters),
                                           ctypes.byref(r)), "df_peak_probe")
        return r.value

    def df_fock(self, h, J, K, D, F, e_one):
        """F = h + J - K / 2 and e_one[0] = tr(D h) on the device."""
        self._check(self.lib.df_fock(self.h, _ptr(h), _ptr(J), _ptr(K), _ptr(D), h.shape[0],
                                     _ptr(F), _ptr(e_one)), "df_fock")

    def df_timing_begin(self, max_calls):
        self._check(self.lib.df_timing_begin(self.h, int(max_calls)), "df_timing_begin")

    def df_timing_end(self):
        """Returns (dict stage -> summed ms, number of timed calls)."""
        ms = (ctypes.c_double * len(STAGES))()
        n = _int()
        self._check(self.lib.df_timing_end(self.h, ms, ctypes.byref(n)), "df_timing_end")
        return dict(zip(STAGES, list(ms))), n.value

    def df_get_status(self):
        return self.lib.df_get_status(self.h)

    def df_debug_build_i32(self, B, b_exp, C, x_sums, k_sums, layout=DF_DENSE, naux=None,
                           nao=None):
        """x_sums int32 [s][naux*nao][nocc], k_sums int32 [s][nb][nao][nao]."""
        naux, nao = _shape(B, layout, naux, nao)
        self._check(self.lib.df_debug_build_i32(self.h, _ptr(B), layout, naux, nao, _ptr(b_exp),
                                                _ptr(C), C.shape[1], _ptr(x_sums), _ptr(k_sums)),
                    "df_debug_build_i32")

    def df_debug_slice_gemm_i32(self, a_dig, b_dig, s, partials):
        _, m, k = a_dig.shape
        n = b_dig.shape[2]
        self._check(self.lib.df_debug_slice_gemm_i32(self.h, _ptr(a_dig), _ptr(b_dig), m, n, k,
                                                     int(s), _ptr(partials)),
                    "df_debug_slice_gemm_i32")


def df_mlp_nparams():
    return load().df_mlp_nparams()


def df_controller_allocate(pred, s_ref, slack=1.0, cost=None):
    """pred: host float array [nblocks][8] of predicted log10 errors; cost: None
    or 8 per-block costs of s = 1..8; returns a list of s."""
    import numpy as np
    p = np.ascontiguousarray(pred, dtype=np.float32)
    nb = p.shape[0]
    out = (ctypes.c_int32 * nb)()
    c = None if cost is None else (ctypes.c_double * 8)(*[float(v) for v in cost])
    rc = load().df_controller_allocate(p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), nb,
                                       int(s_ref), float(slack), c, out)
    if rc != DF_OK:
        raise DFError(rc, "df_controller_allocate: bad arguments")
    return list(out)


def df_prepare_b_size(naux, nao, planes):
    n = ctypes.c_size_t()
    rc = load().df_prepare_b_size(int(naux), int(nao), int(planes), ctypes.byref(n))
    if rc != DF_OK:
        raise DFError(rc, "df_prepare_b_size: bad shape or plane count")
    return n.value


# -- adaptive precision rule (host-only C functions; no context needed) -----------
def df_rule_level(de_rel):
    return load().df_rule_level(float(de_rel))


def df_rule_next_level(level, e_prev, e_now):
    return load().df_rule_next_level(int(level), float(e_prev), float(e_now))


def df_rule_slices(level, fp64_below_level=0):
    return load().df_rule_slices(int(level), int(fp64_below_level))
