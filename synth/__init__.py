"""Seeded synthetic inputs and closed-form problem data (no scheme arithmetic)."""
from .sinsum import (Elastodynamics, Material, SinSum, periodic_moving_solution, plane_wave,
                     stability_test_solution, standing_mms_solution)
from .workloads import (DIRICHLET, batched_instances, PERIODIC, Problem, dt_at_cfl_fraction, gaussian_random_field,
                        grf_problem, node_coords, plane_wave_problem, plane_wave_superposition,
                        poisson_lame, random_material, random_populations, rng,
                        separable_body_table, separable_reference_table,
                        oscillating_walls, separable_table, wall_points,
                        wall_taper)
