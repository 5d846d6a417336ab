"""FP64 CPU oracle for the matrix-free interior eigensolver of arXiv 2012.00217.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product (``paper_2012_00217_amd``) never imports it, and it imports nothing from
the product: the two share no code, tables or constants.  Inputs (disorder
fields, random blocks) are produced by a separate seeded generator module and
handed to both sides as plain arrays.

What the oracle computes, from the definitions in the paper:

* ``basis``       -- the fixed-S^z sector (Sec. 2.1, last paragraph): brute-force
                     enumeration of every L-bit string with the right number of
                     up spins, ascending integer order, and rank lookup by search.
* ``hamiltonian`` -- the sector matrix of eq. (1)/(2) with explicit XX+YY and ZZ
                     couplings and random fields, as a scipy CSR matrix; the
                     shifted block apply ``H X - sigma X``; the diagonal of the
                     spectral fold ``(H - sigma I)^2`` (Sec. 3.2).
* ``spectrum``    -- the nev eigenpairs of H nearest a shift sigma (what LOBPCG on
                     the spectral fold converges to, Sec. 3.2), by dense ``eigh``
                     or shift-invert Lanczos; spectrum bounds.
* ``freefermion`` -- the Delta = 0 closed form (Jordan-Wigner, open chain):
                     many-body energies as subset sums of a tridiagonal matrix's
                     eigenvalues, eigenvectors as Slater determinants.
* ``pcg``         -- the diagonal-(Jacobi-)preconditioned conjugate gradient on
                     the fold, step by step, per column (Sec. 3.2).
* ``linalg``      -- Gram products, Cholesky-QR, residual norms and cluster
                     subspace angles used to compare results.
* ``observables`` -- adjacent gap ratio and half-chain entanglement entropy
                     of eigenpairs (Sec. 2.2).

Conventions where the paper is silent (each is also listed with its reason in
the design notes):

* site i is bit i of the integer state, bit 1 = spin up (S^z = +1/2);
* sector index = number of up spins ``nup = S^z + L/2``;
* states are ordered by ascending integer value;
* ``H = J sum_i [S^x_i S^x_{i+1} + S^y_i S^y_{i+1} + Delta S^z_i S^z_{i+1}]
       + sum_i h_i S^z_i`` on an open chain; J = Delta = 1 is eq. (1).

Every function is pinned by ``tests/test_oracle_*.py`` against values the paper
prints (Table 1), closed forms, an independent tensor-product construction of
eq. (2), or brute force.  Anything not pinned says so in its docstring.
"""

from . import basis, hamiltonian, spectrum, freefermion, pcg, linalg, observables  # noqa: F401
