"""FP64 CPU oracle for the periodic LLG FFT-HSS hot path.

TEST INFRASTRUCTURE ONLY.  This package is the independent, slow, obviously
correct reference against which the HIP library is checked.  Only the test
suite, the smoke check of the package entry point and the CPU-baseline leg of
the benchmark may import it.  The product path (the C-ABI library and its
Python binding) never imports, calls or links anything here, and nothing here
imports the product package: the two share no kernels, helpers, tables or
constant generators.  Seeded inputs come from ``llg_workloads`` (which holds
no arithmetic of the method) or from the caller.

Everything is NumPy / SciPy float64.  Arrays follow one layout throughout: a grid
function is an array of shape (nz, ny, nx) (nz = 1 in two dimensions), a
vector field has shape (3, nz, ny, nx), and a saddle unknown x = (v, r) has
shape (4, nz, ny, nx) with planes v1, v2, v3, r.  Flattened in C order this
is the node index x + nx*(y + ny*z).

Two tiers:
  * ``dense``  -- naive DFT matrices and the assembled saddle matrix, for
    grids of at most a few hundred nodes (checks the FFT tier);
  * everything else -- FFT-based (scipy.fft) matrix-free operators, GMRES,
    the time steppers, energy diagnostics and the midpoint adjoint.

Parity pins for every function live in tests/test_oracle_*.py.
"""

from . import grid, fourier, nodal, operators, dense, gmres, steppers, theory  # noqa: F401
