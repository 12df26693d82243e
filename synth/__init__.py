"""Seeded synthetic inputs shared by the oracle-side tests and the HIP path.

This package generates scenes (triangle meshes with material classes), finds
their specular propagation paths by the image method (done once, on the host,
as the method assumes: fields are calibrated on fixed paths), and packs them
into the interaction-major structure-of-arrays path store that both the FP64
oracle and the GPU library consume.  It holds none of the field arithmetic
(permittivity, Fresnel coefficients, transfer matrices, channel synthesis,
losses): the geometry here only decides *which* paths exist, where they touch
the scene and how long they are.
"""
from .params import Radio, draw_materials, materials_to_raw  # noqa: F401
from .scene import Scene, box_room  # noqa: F401
from .store import PathStore  # noqa: F401
