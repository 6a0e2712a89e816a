"""FP64 CPU oracle for batched state-vector simulation (test infrastructure).

This package is test infrastructure. Only ``tests/``, the smoke check in
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it. The product path (``paper_2509_25075_amd``) never imports, calls or
links anything here, and this package never imports the product.

It is a plain, slow, obviously correct NumPy complex128 simulator written
from the textbook definitions of the operations:

* gates: Pauli rotations R_P(t) = exp(-i t P / 2), Paulis, Hadamard, CNOT, CZ
  (Nielsen & Chuang, *Quantum Computation and Quantum Information*, 2010,
  §4.2 eqs. 4.4-4.6 and §4.3);
* amplitude encoding |x> = x / ||x||_2 and basis-state (zero) initialisation
  (Schuld & Petruccione, *Supervised Learning with Quantum Computers*, 2018,
  §5.2);
* data re-uploading of angle-encoded features (Perez-Salinas et al.,
  *Quantum* 4, 226, 2020);
* Pauli-Z expectation readout, and the fidelity of a quantum autoencoder whose
  trash qubits are reset to |0> (Romero, Olson & Aspuru-Guzik,
  *Quantum Sci. Technol.* 2, 045001, 2017), or measured with only the
  all-zero outcome kept (post-selection, renormalised; Nielsen & Chuang
  §2.2.3, the projective-measurement postulate), or one quantum trajectory of
  the reset channel (the trash qubits measured with an outcome drawn from the
  Born probabilities, then reset; Dalibard, Castin & Molmer, *Phys. Rev.
  Lett.* 68, 580, 1992, for the unravelling of a channel into trajectories);
* mid-circuit channels on one qubit: one trajectory of a Z-basis measurement
  (outcome drawn from the Born probabilities by a given uniform), the state
  renormalised and kept or reset to |0> (Nielsen & Chuang §2.2.3 and §8.3 for
  the measurement and reset channels; trajectories as above), with the
  pathwise cotangent through the renormalisation;
* gradients three ways: the adjoint (reverse state propagation) method
  (Jones & Gacon, arXiv:2009.02823, §3), the parameter-shift rule
  (Mitarai et al., *Phys. Rev. A* 98, 032309, 2018; Schuld et al.,
  *Phys. Rev. A* 99, 032331, 2019, eq. 12) and central finite differences.

Conventions: qubit q is bit q of the amplitude index (little-endian); states
are arrays ``psi[b, i]`` of complex128 with i in [0, 2^n).
"""

from .statevector import (  # noqa: F401
    gate_matrix, apply_1q, apply_cnot, apply_cz, apply_gate, gate_angles,
    encode_amplitude, encode_zero, run_circuit, expz, fidelity_reset,
    fidelity_reset_direct, reset_channel_fidelity_cotangents,
    fidelity_postselect, postselect_fidelity_cotangents, fidelity_postselect_direct,
    trajectory_outcome, fidelity_trajectory, trajectory_fidelity_cotangents,
    fidelity_trajectory_direct, channel_probabilities, apply_channel, channel_cotangent,
)
from .gradients import (  # noqa: F401
    adjoint_vjp, param_shift_theta_jacobian, theta_to_param_grads,
    finite_difference, loss_and_dexpz,
)
