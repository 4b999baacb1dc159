"""Seeded synthetic workloads (inputs only; no method arithmetic)."""
from .cases import (Case, channel_case, refined_cylinder, shear_advection_case, TAG_INLET, TAG_NONE, TAG_OUTLET, TAG_WALL, closed_box,  # noqa: F401
                    cylinder_case, poiseuille_c1, pulsatile_c2, random_blob_case,
                    small_cylinder)
from .serving import GRIDS, Request, request_stream, vessel_case  # noqa: F401,E402
from .aneurysm import aneurysm_case  # noqa: F401,E402
from .aorta import aorta_case, womersley_shapes  # noqa: F401,E402
from .poiseuille import poiseuille_e1, tube_in_box  # noqa: F401,E402
from .moving import PulsatingWall, pulsating_cylinder, pulsating_refined_cylinder  # noqa: F401,E402
