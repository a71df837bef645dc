"""Short-range particle-particle gravity of the split-force N-body method
(Habib et al. 2012, arXiv:1211.4864, Sec. III, Eq. 7) on MI355X (gfx950).

The computation lives in the HIP library ``libhacc_sr.so`` (C ABI declared
in ``include/hacc_sr.h``); this package only marshals arguments to it.
"""
from ._lib import (load, check, strerror, grid_dim, workspace_bytes, bin,
                   rcb_bin, force_rcb, force_vjp_rcb, TIMER_RCB, pm_accel,
                   pm_workspace_bytes, TIMER_PM, full_step,
                   binning_token, force, force_vjp, force_plain, force_vjp_plain, kick, stream,
                   kick_adjoint, count_pairs, timing_enable, timing_read,
                   release_workspace, HaccSrError, EXPORTS, LIB_PATH,
                   TIMER_FORCE, TIMER_VJP, TIMER_BIN, TIMER_WORKLIST,
                   TIMER_FORCE_PLAIN, TIMER_VJP_PLAIN, valu_probe,
                   PROBE_FMA, PROBE_RSQ, PROBE_PAIR_MIX, PROBE_FMAC)


def __getattr__(name):
    # autograd wrappers import torch; load them on first use
    if name in ("SRForce", "sr_force", "SKSRollout", "rollout_sks", "sks_forward"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)


__all__ = ["load", "check", "strerror", "grid_dim", "workspace_bytes", "bin",
           "rcb_bin", "force_rcb", "force_vjp_rcb", "TIMER_RCB", "pm_accel",
           "pm_workspace_bytes", "TIMER_PM", "full_step",
           "binning_token", "force", "force_vjp", "force_plain", "force_vjp_plain", "kick", "stream", "kick_adjoint",
           "count_pairs", "timing_enable", "timing_read", "release_workspace",
           "HaccSrError", "EXPORTS", "LIB_PATH", "SRForce", "sr_force",
           "SKSRollout", "rollout_sks", "sks_forward", "valu_probe", "PROBE_FMA",
           "PROBE_RSQ", "PROBE_PAIR_MIX", "PROBE_FMAC"]
