"""MI355X (gfx950) loop-hafnian library for Gaussian boson sampling.

The loop hafnian of a complex symmetric matrix by the power-trace subset sum
(Quesada et al., arXiv:2010.15595, Sec. IV) and the pure-state photon-number
probability of Sec. II, Eq. (12), the mixed-state probability of Eq. (11)
and the conditional sampling chain of Sec. III, computed by hand-written HIP kernels behind
the C ABI of include/gbs_lhaf.h.  This package is the thin Python binding.
"""
from ._lib import (  # noqa: F401
    BatchPlan,
    GBS_CHARPOLY_EIGEN,
    GBS_CHARPOLY_LABUDDE,
    GBS_DD,
    GBS_FP32_COMP,
    GBS_FP64,
    GbsError,
    MAX_BATCH_DIM,
    MAX_DIM,
    autotune,
    expand,
    finalize,
    haf,
    init,
    lhaf,
    lhaf_device,
    lhaf_device_noalloc,
    lhaf_device_shard,
    combine_partials,
    lhaf_method,
    lhaf_terms,
    lib,
    max_dim,
    pack,
    probability,
    probability_mixed,
    profile_enable,
    profile_read,
    pure_state,
    sample_pure,
    selftest,
    set_layout,
    yardstick_flops,
)
