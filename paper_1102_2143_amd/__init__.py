"""MI355X-native multishift conjugate gradient (HIP for gfx950 behind a C ABI).

Solves (A + sigma_k I) x_k = b for all shifts from one Krylov sequence, for sparse
Hermitian positive-definite A = M^H M (or A given directly).  The numerical work runs in
``libmsc.so``; this package only marshals arguments (see ``api``) and wires the adjoint
into ``torch.autograd`` (see ``autograd``).
"""
from .api import Operator, make_params, solve_batched  # noqa: F401
from ._lib import MscError, load, last_error  # noqa: F401
