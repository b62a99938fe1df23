"""Plain, slow, obviously-correct CPU oracle for randomized QR with column
pivoting (Duersch & Gu, "Randomized QR with Column Pivoting", arXiv 1509.06820).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import or call it.  The product
path (``paper_1509_06820_amd``) never imports it and shares no code with it: no
kernels, helpers, constants or pre/post-processing.

Everything is float64 numpy.  Each function follows one passage of the paper
(section / algorithm / equation named in its docstring) step by step, using a
library matmul or triangular solve only where the paper's own step is a matrix
product.  Readings of passages the paper leaves open are listed in the
docstring of the function that takes them.

Modules
-------
philox       Philox4x64-10 counter-based generator and the Box-Muller map that
             turns its words into the Gaussian compression matrix Omega.
householder  Elementary reflectors and the compact-WY connection matrix T.
qrcp         Sample QRCP, RQRCP (Alg. 4), RSRQRCP (Alg. 5), TRQRCP (Alg. 6),
             unpivoted blocked QR.
svd          TUXV (Alg. 7, any j_max) and the one-sided Jacobi SVD of X.
"""

from .philox import philox4x64_10, omega, uniform52, box_muller  # noqa: F401
from .householder import reflector, apply_reflector, larft, householder_qr, form_q  # noqa: F401
from .qrcp import sample_qrcp, rqrcp, rsrqrcp, trqrcp, unpivoted_qr, sample_update  # noqa: F401
from .svd import tuxv, jacobi_svd  # noqa: F401
