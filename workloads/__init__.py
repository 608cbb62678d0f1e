"""Seeded synthetic inputs for the cut-circuit reconstruction path.

Holds circuit generation, subcircuit simulation (the stand-in for executing the
subcircuit variants on a quantum device) and plain random draws.  It contains
none of the reconstruction arithmetic and is shared by the tests, the benchmark
and the oracle as their common source of inputs.
"""
from .circuits import BridgedChain, CutMap, Subcircuit, bridged_chain
from .entries import circuit_entries, subcircuit_entries
from .configs import (Instance, RECIPES, DD_C4, DD_SCALE, dd_scale_instance, make_instance, config_instance,
                      batch_recipes, batch_instances, dirichlet_target,
                      sample_outputs, random_entries, sample_variant_shots, random_variants)

__all__ = [
    "BridgedChain", "CutMap", "Subcircuit", "bridged_chain", "circuit_entries",
    "sample_variant_shots", "random_variants",
    "subcircuit_entries", "Instance", "RECIPES", "DD_C4", "DD_SCALE", "dd_scale_instance", "make_instance",
    "config_instance", "batch_recipes", "batch_instances", "dirichlet_target",
    "sample_outputs", "random_entries",
]
