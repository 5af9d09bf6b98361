"""Seeded synthetic inputs for the ERBF-fit hot path.

This package builds the *inputs* that both the HIP product path and the CPU
oracle consume: uniform cell-centred grid axes, analytic signed distance
fields sampled on them, band masks, and initial kernel parameters.  It holds
none of the method's arithmetic (no kernel evaluation, no target
normalisation, no loss, no gradient): every function here produces raw data.

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.
"""

from .sdf import (  # noqa: F401
    Primitive,
    sample_sdf,
    random_shape,
    sphere,
    ellipsoid,
    box,
    capsule,
    torus,
)
from .grid import axis_coords, grid_points  # noqa: F401
from .params import (  # noqa: F401
    PARAM_FIELDS,
    random_unit_quaternions,
    init_params_from_points,
    init_params_in_shell,
    pack_params,
    unpack_params,
)
from .configs import (  # noqa: F401
    Problem,
    LevelData,
    make_tiny,
    make_mid,
    make_large,
    make_large_snapshot,
    make_batching,
    make_diff,
    make_custom,
    save_problem,
    load_problem,
)
