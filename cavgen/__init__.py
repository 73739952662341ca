"""Seeded synthetic inputs shared by the oracle and the GPU path.

Holds parameter draws, geometries, velocities and the cavity mode comb only;
no step of the method's arithmetic lives here.
"""
from . import constants
from .params import make_params, draw_sk_tables, PARAM_SEED, TABLE_NAMES
from .systems import make_system, make_cluster, monomer_template, mode_comb, WORKLOADS

__all__ = ["constants", "make_params", "draw_sk_tables", "PARAM_SEED", "TABLE_NAMES",
           "make_system", "make_cluster", "monomer_template", "mode_comb", "WORKLOADS"]
