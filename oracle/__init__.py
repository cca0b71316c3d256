"""FP64 CPU oracle for the Dirac quantum walk of D'Ariano, Mosco, Perinotti and
Tosini, "Discrete Time Dirac Quantum Walk in 3+1 Dimensions".

This package is TEST INFRASTRUCTURE. Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product path (the HIP
library and its Python binding) never does, and shares no code with it.

It is plain, slow and meant to be checked against the paper by eye:

* ``walk``        -- the Weyl/Dirac symbols (Sec. 3.1, 3.2), the lattice
                     geometry, and the position-space transition matrices
                     U_h obtained from the symbol by a small inverse DFT
                     (Sec. 2.1, Fourier representation U_k = sum_h e^{-ik.h} U_h).
* ``stepper``     -- the update rule psi(x,t+1) = sum_h U_h psi(x+h,t)
                     (Sec. 2, update rule and walk operator), applied t times.
* ``dense``       -- the whole walk as a dense (sV x sV) matrix on tiny tori.
* ``fourier``     -- the Fourier evaluation of Sec. 4: DFT with the paper's
                     sign, D_q^t by binary powering, inverse DFT.
* ``states``      -- particle states (Sec. 5.1, Definition 1; Sec. 5.2,
                     particle/antiparticle superposition) and localised states.
* ``observables`` -- norm, position expectation (Sec. 5.2), overlap/fidelity,
                     the drift law (Sec. 5.1) and the k-space Zitterbewegung
                     form of the mean position (Sec. 5.2).
* ``cubic``       -- the cubic-supercell BCC representation of Sec. 4: the
                     two sublattice arrays, the two-sublattice DFT
                     (eq:bcc-dft, eq:bcc-idft) and the evolution through the
                     Cartesian embedding.

Every function names the passage of the paper it follows. Readings of
passages that are ambiguous or garbled are listed in the repository's design
notes and repeated at the function that takes them.
"""
from . import walk, stepper, dense, fourier, states, observables, cubic  # noqa: F401
