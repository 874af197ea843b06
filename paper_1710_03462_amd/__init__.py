"""MI355X (gfx950) SoA/AoS particle-update library: Python binding.

The compute lives in libsoax.so (hand-written HIP kernels behind the C ABI
of include/soax.h); this package marshals torch tensors and streams into
those calls and nothing else.
"""
from ._lib import (AOS, AOS_NAIVE, EULER, EULER_ACC, RK2_ABC, SOA, SoaxError, check,
                   exported_names, lib)
from .autograd import RK2Advect, adjoint, forward_ckpt, rk2_advect, sqdist_loss
from .batch import GRAPH, PER_SET, PERSISTENT, Batch
from .expr import Expr, array, evaluate, maximum, minimum, sqrt
from .particles import ParticleSet, Schema, StepGraph, copy, current_stream, params, probe

Set = ParticleSet  # the name the C ABI's handle goes by

__all__ = ["AOS", "AOS_NAIVE", "EULER", "EULER_ACC", "RK2_ABC", "SOA", "SoaxError", "check",
           "exported_names", "lib", "RK2Advect", "adjoint", "forward_ckpt", "rk2_advect",
           "sqdist_loss", "GRAPH", "PER_SET", "PERSISTENT", "Batch", "ParticleSet", "Schema",
           "copy", "current_stream", "params", "probe", "Set", "StepGraph", "Expr", "array", "evaluate", "maximum", "minimum",
           "sqrt"]
