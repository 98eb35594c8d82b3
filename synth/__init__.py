"""Seeded synthetic inputs shared by the oracle tests, the HIP path and the benchmark."""
from .workloads import (Workload, BatchInstance, slab_1d, slab_1d_two_tau, slab_1d_multiscale,
                        uniform_field_1d, cavity_2d, two_material_2d, batch_instances,
                        batch_workloads, gaussian_source, AdjointCase, adjoint_case,
                        slab_1d_bands, sine_dispersion_bands, nongray_two_material_2d,
                        seeded_temperature)

__all__ = ["Workload", "BatchInstance", "slab_1d", "slab_1d_two_tau", "slab_1d_multiscale",
           "uniform_field_1d", "cavity_2d", "two_material_2d", "batch_instances",
           "batch_workloads", "gaussian_source", "AdjointCase", "adjoint_case",
           "slab_1d_bands", "sine_dispersion_bands", "nongray_two_material_2d",
           "seeded_temperature"]
