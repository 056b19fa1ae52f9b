"""MI355X-native auxiliary Kalman MCMC (parallel-in-time filter and sampler).

The sampler itself lives in the HIP library libauxkf.so (include/akf.h); this
package is its Python binding.  Importing the package does not load the
library; the first call does, and fails loudly if it has not been built.
"""
from .workloads import (EMIT_GAUSSIAN, EMIT_POISSON_LOG, EMIT_STUDENT_T,  # noqa: F401
                        EMIT_STOCH_VOL, EMIT_MVT)


def __getattr__(name):
    # lazy: the binding imports torch and loads the HIP library on first use
    if name in ("DeviceModel", "Workspace", "mh_step", "mh_step_noalloc", "mh_run",
                "aux_filter", "rts_sample", "dnc_sample", "sqrt_filter_sample", "smoother",
                "LGSSM", "lgssm_loglik", "lgssm_loglik_grad", "KalmanLogLik", "BatchPlan",
                "GibbsState", "gibbs_init", "gibbs_sweep", "n_theta", "ST_FWD_NOT_PD",
                "ST_REV_NOT_PD", "ST_NONFINITE"):
        from . import sampler
        return getattr(sampler, name)
    raise AttributeError(name)
