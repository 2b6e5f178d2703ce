"""FP64 CPU oracle for the T-product of third-order quaternion tensors.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the GPU path (no kernels, tables,
helpers or pre/post-processing); the only thing both sides consume is the
seeded input generator in ``synth``, which holds no T-product arithmetic.

What it computes is the plain definition of the T-product
(Section 2.4, Definition of the T-product):

    A * B := fold( bcirc(A) . unfold(B) ),

with quaternion matrix products built from Hamilton's rules
(i^2 = j^2 = k^2 = ijk = -1, ij = k, jk = i, ki = j; Section 1 and Section 2.2).
Everything is float64 numpy.  Tensors use the layout (4, p, rows, cols):
plane c is the c-th real component (a, b, c, d) of a + b i + c j + d k, face k
is X[:, k].

Modules
-------
quaternion : element and matrix algebra (Hamilton product, conjugates).
tproduct   : bcirc / unfold / fold, the definitional T-product, its sampled
             entries, the tensor conjugate transpose, identity tensor, the
             least-squares loss and its adjoints, error norms.
fast       : the paper's FFT-based Algorithm 5.1 in FP64 (the CPU FFT-based
             version the benchmark times; pinned against the definition).
tsvd       : the quaternion t-SVD A = U * S * V^H built on the frequency-pair
             matrices that Theorem 5.1 makes multiplicative, and the singular
             values of bcirc(A) from the definition.
"""
from .fast import tprod_fft  # noqa: F401
from . import tsvd  # noqa: F401  (module: tsvd.tsvd, tsvd.bcirc_singular_values)
from .quaternion import qmul, qmatmul, qconj, qconjT, qnorm2  # noqa: F401
from .tproduct import (  # noqa: F401
    bcirc,
    unfold,
    fold,
    tprod,
    tprod_faces,
    tprod_rows,
    tprod_cols,
    tprod_entries,
    tconjT,
    identity,
    loss,
    adjoints,
    rel_frob,
)
