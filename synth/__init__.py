"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module only draws random inputs: degree-corrected stochastic block model
graphs shaped like the static and streaming partition workloads the paper
measures on (Section III, Table I shapes), Gaussian starting blocks (Section III,
random initialisation), the uniform draws consumed by k-means++ seeding, and the
emerging-edge / snowball stage streams (Section III, streaming warm starts).
It contains none of the method's arithmetic: no Laplacian, no eigensolver, no
clustering.  Everything is a deterministic function of the seed (numpy's
counter-based Philox generator).
"""
from .sbm import (SBMGraph, dcsbm, block_sizes, gaussian_block, kmeans_draws,
                  emerging_stages, snowball_stages)
from .configs import CONFIGS, config

__all__ = ["SBMGraph", "dcsbm", "block_sizes", "gaussian_block", "kmeans_draws",
           "emerging_stages", "snowball_stages", "CONFIGS", "config"]
