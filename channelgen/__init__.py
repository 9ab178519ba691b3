"""Seeded synthetic XL-MIMO channel generator shared by the oracle tests, the GPU
tests and the benchmark.

It only draws inputs -- channels, regularisation values and request streams --
and holds none of the precoder's arithmetic (no Gram, no solve, no precoder).
"""

from .xlmimo import (  # noqa: F401
    WORKLOADS,
    Workload,
    workload,
    channel_batch,
    channel_instance,
    xi_from_snr,
    serving_requests,
    request_channels,
    instance_matrix,
    device_pool,
    device_pool_r,
    block_channel_instance,
    block_channel_batch,
    vr_order,
    vr_spans,
    sorted_channel_batch,
)
