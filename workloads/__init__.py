"""Seeded synthetic workloads for hard-coded-gradient GRAPE.

This package only *generates inputs*: superconducting-circuit operators
(transmons, cavities), control amplitudes, initial states, Haar-random target
unitaries and forbidden-level projectors.  It holds none of the method's
arithmetic (no propagation, no cost, no gradient), so both the FP64 oracle and
the GPU path can be fed from it without sharing any computation.

The physical systems follow the benchmark families of the paper: a driven
transmon coupled to a cavity (Sec. IV.B, Hamiltonian H_1) and coupled
transmons (Sec. IV.B, Hamiltonian H_2), written in the bare product basis with
the cavity index running fastest.  Units: rad/ns for energies, ns for time,
hbar = 1.
"""
from .circuits import (destroy, number, embed, transmon_cavity_system,
                       two_transmon_cavity_system, three_transmon_chain, haar_unitary, Problem)
from .configs import CONFIGS, make_config, serving_stream, problem_summary

__all__ = ["destroy", "number", "embed", "transmon_cavity_system",
           "two_transmon_cavity_system", "three_transmon_chain", "haar_unitary", "Problem",
           "CONFIGS", "make_config", "serving_stream", "problem_summary"]
