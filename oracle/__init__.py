"""Plain FP64 CPU oracle for the nested shift-invert diagonalization of the
random-field Heisenberg chain (Kutsuzawa & Todo, arXiv:2203.09732).

TEST INFRASTRUCTURE ONLY. This package is imported by ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` and
by nothing else. It shares no code with the HIP library: no kernels, headers,
tables, helpers or constants. It imports nothing from the product package.

Every routine is a slow, direct statement of what the paper defines:

* ``model``    - Eq. (1) in the S^z basis of the S^z = 0 sector, built by
                 filtering all 2^L states, plus an independent Kronecker-product
                 construction used to pin it;
* ``precond``  - the Jacobi and row-norm diagonal preconditioners (Sec. II);
* ``minres``   - preconditioned MINRES in the order of Alg. 2 (App. A);
* ``lanczos``  - shift-invert Lanczos in the order of Alg. 1, with full
                 reorthogonalisation against the earlier basis vectors
                 (Fig. 1 caption), and the dense-eigensolver definition of the
                 eigenpairs nearest sigma;
* ``twist``    - the twist overlap z = <psi|U_twist|psi> (Sec. III, App. B);
* ``adjoint``  - Hellmann-Feynman energies' derivatives and eigenvector
                 derivatives by the first-order perturbation sum;
* ``observables`` - the bipartite entanglement entropy (Schmidt
                 decomposition) and the level-spacing ratio (Sec. IV).

Conventions fixed here (the paper leaves them open): site j = 1..L is bit
j-1 of the state integer, a set bit is S^z = +1/2, the basis is in ascending
integer order, J = 1.
"""
from . import model, precond, minres, lanczos, twist, adjoint, observables  # noqa: F401
