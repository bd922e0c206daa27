"""FP64 CPU oracle for signal-whitened FFT window matching (SWiFT-IR).

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this package.  It shares no code with
the HIP path and the product path never calls it.
"""
from .swift_oracle import (  # noqa: F401
    Params,
    gather,
    taper_1d,
    taper_2d,
    prepare,
    whitened_surface,
    peak_stats,
    match_pair,
    match_grad,
    project,
    pyramid,
    fit_affine,
    level_to_base,
    base_to_level,
    apply_affine,
    render,
    stack_windows,
    correspondence,
    match_weight,
    fit_section,
    refine_step,
    centroid_jacobian,
    surface_hessian,
    mesh_node_xy,
    mesh_triangles,
    mesh_band,
    mesh_triangle_of,
    fit_mesh,
    render_mesh,
    render_mesh_at,
    mesh_windows,
    pearson_surface,
    pearson_peak,
    pearson_pair,
)
