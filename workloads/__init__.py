"""Seeded synthetic neuron workloads shared by the oracle, the tests and the bench.

This package only draws random neurons (shapes, weights, biases, thresholds,
fan-in index sets).  It holds none of the enumeration arithmetic, so both the
CPU oracle and the HIP path can consume its output without sharing any code
that computes a truth table.
"""
from .gen import (  # noqa: F401
    CONFIG_SEED_BASE,
    NeuronSet,
    make_config,
    cfg0,
    cfg1,
    cfg2,
    cfg3,
    cfg4_train,
    cfg4_screen,
    random_neurons,
    mlp_init,
    subset,
    concat,
    network_fanin,
    tseitin_instances,
)
