"""Seeded synthetic workloads: circuit descriptors and input tensors.

This package is pure data generation. It holds none of the simulation
arithmetic: it only lays out gate lists (which gate acts on which qubit with
which parameter index) and draws seeded random numbers. Both the FP64 oracle
(``oracle/``) and the HIP path (``paper_2509_25075_amd``) consume what it
produces, and neither imports the other.
"""

from .circuits import (  # noqa: F401
    GATE_DTYPE, OP, OP_NAMES, ROTATIONS, Circuit, concat, inverse_structure,
    hea_ry_rz_ring, rxyz_cz_ring, reupload_ry_rz_chain, ry_rz_chain,
    random_circuit,
)
from .data import (  # noqa: F401
    WORKLOADS, Workload, make_workload, amplitude_inputs, uniform_params,
    pm1_labels, uniform_features, upstream_weights, uneven_batch_spec,
    UnevenBatch, uneven_batch,
)
