"""mdgemm: mixed-datatype matrix multiplication on MI355X (gfx950).

C := beta*C + alpha*op(A)*op(B) with A, B and C independently stored as
s/d/c/z and a separately chosen computation precision (Van Zee, Parikh,
van de Geijn, "Supporting mixed-datatype matrix multiplication within the
BLIS framework").  The product runs in the HIP kernels of libmdgemm.so; this
package only marshals torch tensors into its C ABI.
"""
from .api import gemm, plan, grouped, GroupedCall, dt_of, MdgemmError  # noqa: F401
