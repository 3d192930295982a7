"""Seeded synthetic inputs shared by the GPU library's tests/bench and the CPU oracle.

This package draws random numbers and builds input arrays only: EM-like uint8
volumes, He-normal weight vectors, layer specifications, tile lists and patch
draws. It contains none of the network arithmetic (no convolution, pooling,
activation or loss), so neither side of a parity test borrows computation from
the other through it.
"""
from .em import em_slice, em_volume  # noqa: F401
from .nets import (  # noqa: F401
    NET_A, NET_B, NET_S, NETS, conv_layers, he_normal_params, random_bias_params,
    calibrated_params, param_count, load_calibration,
)
from .workloads import (  # noqa: F401
    CONFIGS, batch_tiles, student_patch_origins, mixed_difficulty_volume, maskextend_maps,
)
