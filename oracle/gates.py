"""Gate matrices in complex128.

T is diag(1, (1+i)/sqrt 2) (Sec. 2.4, below Eq. 3); CZ is diag(1, 1, 1, -1)
(Sec. 2.4, below Eq. 5); P0 = diag(1, 0), P1 = diag(0, 1) and Z = diag(1, -1)
(Sec. 2.1, Eq. 1).  The paper's "X" and "Y" gates of the random circuits are
read as the principal square roots of X and Y (its Ref. [6]); H is the
Hadamard gate of the first layer.

Controlled gates follow Supp. Eq. 1: a controlled-U on (control, target) is
P0 x I + P1 x U, the projector on the control and U^b on the target; CZ is
the case U = Z, CNOT the case U = X, and CY the case U = Y (Pauli X and Y).
"""

import numpy as np

SQ2 = np.sqrt(2.0)

H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / SQ2
SX = 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128)
SY = 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]], dtype=np.complex128)
T = np.array([[1, 0], [0, (1 + 1j) / SQ2]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
CZ = np.diag(np.array([1, 1, 1, -1], dtype=np.complex128))
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)

# the U of each controlled two-qubit gate (qubits listed control first)
CONTROLLED_U = {"cz": Z, "cx": X, "cy": Y}

ONE_QUBIT = {"h": H, "sx": SX, "sy": SY, "t": T}
DIAGONAL = {"t"}
