"""Surfel radiosity transport on AMD Instinct MI355X (gfx950).

The HIP library libgsrad.so (C ABI in include/gsrad.h) holds every kernel;
``paper_2509_18497_amd.gsrad`` is its Python binding.
"""
from . import gsrad  # noqa: F401
from .gsrad import (BF16, BVH, FF, FP32, Batch, GsradError, RadiosityFn, Tape, batch_create,  # noqa: F401
                    batch_transport_backward, batch_transport_solve, build_bvh, check, check_reciprocity, direct_light,
                    effective_area, ff_dense, ff_from_csr, form_factors, opacity_backward, profile_enable, profile_report,
                    ray_hits, reflectance, tape_grad_F_dense, transport_backward, transport_solve, transport_solve_noalloc,
                    version, brdf_reflectance, brdf_backward, direct_light_sh, transport_solve_sh,
                    transport_backward_sh, batch_set_lanes, batch_set_precision, ff_center, ff_center_backward,
                    geometry_backward, direct_light_backward, MC, mc_create, mc_estimate, mc_solve)
