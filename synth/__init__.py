"""Seeded synthetic F-engine frames for the X-engine and its oracle.

This package only draws random numbers and packs them into the 4+4-bit
offset-binary sample bytes that an F-engine emits (Sec. II-A, the footnote on
offset encoding).  It holds none of the correlator's arithmetic: no decode, no
products, no sums.  Both the HIP path and the CPU oracle take their inputs from
here, so that the two sides see the same bytes.
"""

from .frames import (  # noqa: F401
    WORKLOADS,
    Workload,
    batch_frame,
    batch_instances,
    encode,
    gen_channel,
    gen_frame,
    frame_sha256,
    stream_frame,
    workload,
)
from .beams import gen_beam_weights  # noqa: F401
from .flags import gen_flags, pack_flags, unpack_flags  # noqa: F401
