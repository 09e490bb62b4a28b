"""Seeded synthetic inputs (boundary nodes, A, right-hand sides) shared by the
tests, the benchmark and the CPU oracle. Holds no solver arithmetic."""
from . import geometry
from .configs import (Domain, SEED, annulus, batch_domain, config3, circles_unbounded, closed_form_rhs, config0,
                      config1, config2, close_shapes, config4, disk, domain_from_fourier, example2_circles,
                      example4_circles, exterior_points_fourier, fourier_perturbed_circles,
                      interior_points_config1)

__all__ = ["geometry", "Domain", "SEED", "annulus", "batch_domain", "config3", "circles_unbounded", "closed_form_rhs",
           "config0", "config1", "config2", "close_shapes", "config4", "disk", "domain_from_fourier", "example2_circles",
           "example4_circles", "exterior_points_fourier", "fourier_perturbed_circles", "interior_points_config1"]
