"""phi4pmc: particle Monte Carlo samplers for 2D lattice phi^4 on MI355X.

Thin Python binding of ``libphi4pmc.so`` (see ``include/phi4pmc.h``).  The
functions below carry the C names and only marshal arguments: device buffers
are torch tensors on a HIP device, every step of the samplers runs in the
library's HIP kernels.  There is no CPU fallback: if the library is missing
or no GPU is present, calls raise.
"""

import ctypes
import math
import os

from . import _abi
from ._abi import (  # noqa: F401
    PHI4_OK, PHI4_DONE, PHI4_EINVAL, PHI4_EHIP, PHI4_ECHOL, PHI4_ENONFINITE,
    PHI4_FP32, PHI4_BF16, PHI4_FP16, PHI4_INIT, PHI4_PROPOSE, PHI4_ACCEPT,
    PHI4_RESAMPLE, PHI4_NS_PICK, PHI4_MAX_SITES, PHI4_KERNEL_RW, PHI4_KERNEL_IRMH, PHI4_KERNEL_HMC,
    PHI4_IRMH_MAX_SITES, KERNELS, PHI4_NS_RW, PHI4_NS_SLICE, PHI4_SLICE, NS_KERNELS, Phi4Error,
    SmcConfig, NsConfig, lib, library_path,
)

PRECISIONS = {"fp32": PHI4_FP32, "bf16": PHI4_BF16, "fp16": PHI4_FP16}


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check(rc, name):
    if rc < 0:
        raise Phi4Error(rc, f"{name}: {lib().phi4_last_error().decode()}")
    return rc


def _require_cuda(*tensors):
    for t in tensors:
        if t is not None and not t.is_cuda:
            raise ValueError("phi4pmc needs device tensors (torch.cuda / HIP)")


def _workspace(nbytes, device):
    import torch
    # 256 extra bytes so the carve start can be aligned to 256
    raw = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw, raw[off:off + int(nbytes)]


# --------------------------------------------------------------- samplers

def smc_workspace_bytes(cfg):
    return int(lib().smc_workspace_bytes(ctypes.byref(cfg)))


def smc_init(cfg, phi, S, workspace, stream=None):
    _require_cuda(phi, S, workspace)
    h = ctypes.c_void_p()
    _check(lib().smc_init(ctypes.byref(cfg), _ptr(phi), _ptr(S), _ptr(workspace),
                          ctypes.c_size_t(workspace.numel()), _stream(stream),
                          ctypes.byref(h)), "smc_init")
    return h


def smc_restart(h, seed, run=0):
    _check(lib().smc_restart(h, ctypes.c_uint32(seed), ctypes.c_uint32(run)), "smc_restart")


def smc_reweight_resample(h, sync=True):
    beta = ctypes.c_double(math.nan)
    rc = _check(lib().smc_reweight_resample(h, ctypes.byref(beta) if sync else None),
                "smc_reweight_resample")
    return rc, beta.value


def smc_mutate(h, sync=True):
    acc = ctypes.c_double(math.nan)
    rc = _check(lib().smc_mutate(h, ctypes.byref(acc) if sync else None), "smc_mutate")
    return rc, acc.value


def smc_run(h, max_levels=100000):
    levels = ctypes.c_int32(0)
    rc = _check(lib().smc_run(h, ctypes.c_int32(max_levels), ctypes.byref(levels)), "smc_run")
    return rc, levels.value


def smc_batch_run(handles, max_levels=100000, stream=None):
    """Advance many SMC handles together (one replayed hipGraph per pair of
    levels); returns (rc, levels per run)."""
    n = len(handles)
    arr = (ctypes.c_void_p * n)(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                  for h in handles])
    levels = (ctypes.c_int32 * n)()
    rc = _check(lib().smc_batch_run(arr, ctypes.c_int32(n), ctypes.c_int32(max_levels), levels,
                                    _stream(stream)), "smc_batch_run")
    return rc, list(levels)


def ns_workspace_bytes(cfg):
    return int(lib().ns_workspace_bytes(ctypes.byref(cfg)))


def ns_init(cfg, phi, S, workspace, stream=None):
    _require_cuda(phi, S, workspace)
    h = ctypes.c_void_p()
    _check(lib().ns_init(ctypes.byref(cfg), _ptr(phi), _ptr(S), _ptr(workspace),
                         ctypes.c_size_t(workspace.numel()), _stream(stream),
                         ctypes.byref(h)), "ns_init")
    return h


def ns_step(h, sync=True):
    done = ctypes.c_int32(0)
    rc = _check(lib().ns_step(h, ctypes.byref(done) if sync else None), "ns_step")
    return rc, bool(done.value)


def logz(h):
    z, se = ctypes.c_double(), ctypes.c_double()
    _check(lib().logz(h, ctypes.byref(z), ctypes.byref(se)), "logz")
    return z.value, se.value


OBSERVABLE_NAMES = ("mean_abs_m", "beta_or_logX", "acc", "eps", "levels",
                    "dbeta_or_sstar", "ess_or_H", "tau", "solve_iters", "done")


def phi4_observables(h):
    out = (ctypes.c_double * 10)()
    _check(lib().phi4_observables(h, out), "phi4_observables")
    return dict(zip(OBSERVABLE_NAMES, list(out)))


SWEEPS = {"auto": 0, "fused": 1, "passes": 2}


def phi4_tile_choice(n, d, precision="fp32"):
    """(particles, columns, threads) of the tuned proposal-product tile, zeros if untimed."""
    rows, cols, threads = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().phi4_tile_choice(n, d, PRECISIONS[precision], ctypes.byref(rows),
                                  ctypes.byref(cols), ctypes.byref(threads)), "phi4_tile_choice")
    return rows.value, cols.value, threads.value


def phi4_set_tile(n, d, precision, rows, cols, threads=256):
    _check(lib().phi4_set_tile(n, d, PRECISIONS[precision], rows, cols, threads),
           "phi4_set_tile")


def phi4_set_sweep(h, form="auto"):
    _check(lib().phi4_set_sweep(h, ctypes.c_int32(SWEEPS[form])), "phi4_set_sweep")


def phi4_set_timing(h, enabled=True):
    _check(lib().phi4_set_timing(h, ctypes.c_int32(1 if enabled else 0)), "phi4_set_timing")


def phi4_kernel_time(h):
    ms, n = ctypes.c_double(), ctypes.c_int32()
    _check(lib().phi4_kernel_time(h, ctypes.byref(ms), ctypes.byref(n)), "phi4_kernel_time")
    return ms.value, n.value


def phi4_destroy(h):
    if h is not None and h.value:
        lib().phi4_destroy(h)


# ------------------------------------------------------------- step level

def phi4_step_workspace_bytes(n, d):
    return int(lib().phi4_step_workspace_bytes(ctypes.c_int32(n), ctypes.c_int32(d)))


def phi4_normals(seed, run, level, step, purpose, n, d, out, rows=None, stream=None):
    _require_cuda(out, rows)
    _check(lib().phi4_normals(ctypes.c_uint32(seed), ctypes.c_uint32(run), ctypes.c_int32(level),
                              ctypes.c_int32(step), ctypes.c_int32(purpose), _ptr(rows),
                              ctypes.c_int32(n), ctypes.c_int32(d), _ptr(out), _stream(stream)),
           "phi4_normals")


def phi4_action(phi, N, L, m2, lam, S, absM=None, stream=None):
    _require_cuda(phi, S, absM)
    _check(lib().phi4_action(_ptr(phi), ctypes.c_int32(N), ctypes.c_int32(L), ctypes.c_double(m2),
                             ctypes.c_double(lam), _ptr(S), _ptr(absM), _stream(stream)),
           "phi4_action")


def phi4_resample_systematic(w, N, U, ancestors, workspace, stream=None):
    _require_cuda(w, ancestors, workspace)
    _check(lib().phi4_resample_systematic(_ptr(w), ctypes.c_int32(N), ctypes.c_uint32(U),
                                          _ptr(ancestors), _ptr(workspace),
                                          ctypes.c_size_t(workspace.numel()), _stream(stream)),
           "phi4_resample_systematic")


def phi4_reweight(S, N, beta, ess_frac, workspace, w=None, stream=None):
    _require_cuda(S, workspace, w)
    out = (ctypes.c_double * 4)()
    _check(lib().phi4_reweight(_ptr(S), ctypes.c_int32(N), ctypes.c_double(beta),
                               ctypes.c_double(ess_frac), _ptr(w), out, _ptr(workspace),
                               ctypes.c_size_t(workspace.numel()), _stream(stream)),
           "phi4_reweight")
    return dict(dbeta=out[0], beta=out[1], dlogz=out[2], ess=out[3])


def phi4_covariance(phi, N, d, sigma, workspace, rows=None, stream=None):
    _require_cuda(phi, sigma, workspace, rows)
    _check(lib().phi4_covariance(_ptr(phi), _ptr(rows), ctypes.c_int32(N), ctypes.c_int32(d),
                                 _ptr(sigma), _ptr(workspace), ctypes.c_size_t(workspace.numel()),
                                 _stream(stream)), "phi4_covariance")


def phi4_whiten_workspace_bytes(n, d):
    return lib().phi4_whiten_workspace_bytes(ctypes.c_int32(n), ctypes.c_int32(d))


def phi4_whiten(phi, N, d, L, r, workspace, rows=None, mu=None, stream=None):
    _require_cuda(phi, L, r, workspace, rows, mu)
    _check(lib().phi4_whiten(_ptr(phi), _ptr(rows), ctypes.c_int32(N), ctypes.c_int32(d), _ptr(L),
                             _ptr(r), _ptr(mu), _ptr(workspace), ctypes.c_size_t(workspace.numel()),
                             _stream(stream)), "phi4_whiten")


def phi4_slice_move(phi, n, L, m2, lam, s_star, prior_var, seed, run, level, step, dirs, S,
                    rows=None, absM=None, stream=None):
    _require_cuda(phi, dirs, S, rows, absM)
    _check(lib().phi4_slice_move(_ptr(phi), _ptr(rows), _ptr(dirs), ctypes.c_int32(n),
                                 ctypes.c_int32(L), ctypes.c_double(m2), ctypes.c_double(lam),
                                 ctypes.c_double(s_star), ctypes.c_double(prior_var),
                                 ctypes.c_uint32(seed), ctypes.c_uint32(run), ctypes.c_int32(level),
                                 ctypes.c_int32(step), _ptr(S), _ptr(absM), _stream(stream)),
           "phi4_slice_move")


def phi4_cholesky(sigma, d, L, workspace, stream=None):
    _require_cuda(sigma, L, workspace)
    tau = ctypes.c_double()
    _check(lib().phi4_cholesky(_ptr(sigma), ctypes.c_int32(d), _ptr(L), ctypes.byref(tau),
                               _ptr(workspace), ctypes.c_size_t(workspace.numel()),
                               _stream(stream)), "phi4_cholesky")
    return tau.value


def phi4_mutate(src, dst, n, L, m2, lam, Bt, kind, beta, s_star, prior_var, seed, run, level,
                step0, n_steps, zsign, precision, S, absM=None, acc_count=None, acc_flags=None,
                prop=None, rows=None, workspace=None, stream=None):
    _require_cuda(src, dst, Bt, S, absM, acc_count, acc_flags, prop, rows, workspace)
    raw = None
    if workspace is None and L * L > 256:
        raw, workspace = _workspace(phi4_step_workspace_bytes(n, L * L), src.device)
    wbytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().phi4_mutate(_ptr(src), _ptr(dst), _ptr(rows), ctypes.c_int32(n), ctypes.c_int32(L),
                             ctypes.c_double(m2), ctypes.c_double(lam), _ptr(Bt), ctypes.c_int32(kind),
                             ctypes.c_double(beta), ctypes.c_double(s_star),
                             ctypes.c_double(prior_var), ctypes.c_uint32(seed), ctypes.c_uint32(run),
                             ctypes.c_int32(level), ctypes.c_int32(step0), ctypes.c_int32(n_steps),
                             ctypes.c_float(zsign), ctypes.c_int32(precision), _ptr(S), _ptr(absM),
                             _ptr(acc_count), _ptr(acc_flags), _ptr(prop), _ptr(workspace),
                             ctypes.c_size_t(wbytes), _stream(stream)),
           "phi4_mutate")
    del raw


# ------------------------------------------------------ run-level helpers

class SMC:
    """One adaptive tempered SMC run with torch-owned device buffers."""

    def __init__(self, L, N, m2, lam, ess_frac=0.5, n_steps=10, acc_target=None, eps0=0.0,
                 seed=0, run=0, precision="fp32", sweep="auto", device="cuda", kernel="rw",
                 n_leapfrog=20):
        import torch
        if acc_target is None:   # HMC is steered to a higher acceptance than the random walk
            acc_target = 0.65 if kernel == "hmc" else 0.3
        self.cfg = SmcConfig(L=L, N=N, m2=m2, lambda_=lam, ess_frac=ess_frac, n_steps=n_steps,
                             acc_target=acc_target, eps0=eps0, seed=seed, run=run,
                             precision=PRECISIONS[precision], kernel=KERNELS[kernel],
                             n_leapfrog=n_leapfrog)
        nbytes = smc_workspace_bytes(self.cfg)
        if nbytes == 0:
            raise Phi4Error(PHI4_EINVAL, "invalid SMC configuration")
        self.d = L * L
        self.phi = torch.empty((N, self.d), dtype=torch.float32, device=device)
        self.S = torch.empty(N, dtype=torch.float32, device=device)
        self._raw, self.workspace = _workspace(nbytes, device)
        self.h = smc_init(self.cfg, self.phi, self.S, self.workspace)
        if sweep != "auto":
            phi4_set_sweep(self.h, sweep)

    def run(self, max_levels=10000):
        return smc_run(self.h, max_levels)

    def restart(self, seed, run=0):
        smc_restart(self.h, seed, run)

    def logz(self):
        return logz(self.h)[0]

    def observables(self):
        return phi4_observables(self.h)

    def close(self):
        phi4_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                self.close()
        except Exception:
            pass


class NS:
    """One nested-sampling run with torch-owned device buffers."""

    def __init__(self, L, n_live, k_delete, n_steps, m2, lam, prior_var=4.0, term_frac=1e-3,
                 acc_target=0.3, eps0=0.0, seed=0, run=0, precision="fp32", sweep="auto",
                 device="cuda", kernel="rw"):
        import torch
        self.cfg = NsConfig(L=L, n_live=n_live, k_delete=k_delete, n_steps=n_steps, m2=m2,
                            lambda_=lam, prior_var=prior_var, term_frac=term_frac,
                            acc_target=acc_target, eps0=eps0, seed=seed, run=run,
                            precision=PRECISIONS[precision], kernel=NS_KERNELS[kernel])
        nbytes = ns_workspace_bytes(self.cfg)
        if nbytes == 0:
            raise Phi4Error(PHI4_EINVAL, "invalid nested-sampling configuration")
        self.d = L * L
        self.phi = torch.empty((n_live, self.d), dtype=torch.float32, device=device)
        self.S = torch.empty(n_live, dtype=torch.float32, device=device)
        self._raw, self.workspace = _workspace(nbytes, device)
        self.h = ns_init(self.cfg, self.phi, self.S, self.workspace)
        if sweep != "auto":
            phi4_set_sweep(self.h, sweep)

    def run(self, max_iter=1000000, sync_every=8):
        it = 0
        while it < max_iter:
            it += 1
            sync = it % sync_every == 0
            rc, done = ns_step(self.h, sync=sync)
            if sync and done:
                break
        ns_step(self.h, sync=True)   # returns at once if done, else one more step
        z, se = logz(self.h)
        return z, se

    def observables(self):
        return phi4_observables(self.h)

    def close(self):
        phi4_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                self.close()
        except Exception:
            pass
