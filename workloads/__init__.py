"""Seeded synthetic inputs for the Monte Carlo direct-illumination hot path.

This package produces meshes, environment maps, cameras and G-buffers that
both the CPU oracle and the HIP path consume.  It contains none of the
estimator's arithmetic: no sampling, no BSDF, no MIS, no shadow rays.  The
G-buffer is made by casting primary rays against the *analytic* surfaces the
meshes tessellate (primary visibility is an input to the method, not part of
it).

Every generator is deterministic given its numpy PCG64 seed.
"""

from .configs import Workload, make_workload, from_arrays, upstream_grads, noisy_lighting, CONFIGS  # noqa: F401
