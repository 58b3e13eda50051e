"""MI355X-native boundary-MPS maximum-likelihood coset decoding.

The contraction runs in ``libtnmld.so`` (HIP, gfx950); this package only
marshals arguments.  See include/tnmld.h for the C ABI.
"""
from ._lib import TNError, lib, LIB_PATH  # noqa: F401
from .api import (SegmentInput, SegmentOutput, bitflip_plan_info, check_input_values, code_stabilizers,  # noqa: F401
                  coset_loglik, coset_loglik_backward, coset_loglik_backward_saved, coset_loglik_save, decode,
                  decode_bitflip, decode_bitflip_segments, decode_rounds, decode_segments, log_posterior, plan_info,
                  set_tuning, states_bytes, workspace_bytes)
from .fit import fit_log_rates  # noqa: F401

from . import tune as _tune  # noqa: E402

try:  # apply the autotuner's cached launch shapes (needs only the host library)
    _tune.load(apply=True)
except Exception:  # a missing or unreadable cache keeps the defaults
    pass

__all__ = ["TNError", "SegmentInput", "SegmentOutput", "coset_loglik", "coset_loglik_backward", "coset_loglik_save",
           "coset_loglik_backward_saved", "states_bytes", "log_posterior", "decode", "decode_segments",
           "decode_rounds", "decode_bitflip", "decode_bitflip_segments", "bitflip_plan_info", "check_input_values",
           "workspace_bytes", "fit_log_rates", "plan_info", "set_tuning", "code_stabilizers", "lib", "LIB_PATH"]
