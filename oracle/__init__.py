"""CPU oracle for the cyclic-group RAID-6 code (Jackson, Rumynin, Zaboronski,
"An approach to RAID-6 based on cyclic groups").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what the GPU library computes.  It exists so that the
tests, the smoke check in ``__graft_entry__`` and the CPU-baseline leg of
``bench.py`` can check the GPU results.  The product library never imports,
links or calls it, and it shares no code with the HIP kernels.

Data layout (shared with the library only as a convention, not as code):
a *strip* is ``p-1`` rows of ``W`` bytes, row ``r`` holding the coefficient of
``x^r``.  Bit ``b`` of byte ``j`` across the rows of a strip is one ring
element, so every operation acts on whole rows with XOR.  A stripe is ``k``
data strips ``D_0 .. D_{k-1}`` followed by ``P`` (index ``k``) and ``Q``
(index ``k+1``).

Modules:

* :mod:`oracle.ring` -- the ring F2[x]/(1+x+...+x^(p-1)) acted on by the
  Sylvester matrix S_p (Lemma 3.4.1).
* :mod:`oracle.zp_raid` -- Z_p-RAID encode and recovery of one or two erased
  strips (Corollary 3.2.4, Lemma 3.1.2, Sections 4.3 and 4.6).
* :mod:`oracle.rs_gf256` -- the conventional Reed-Solomon P+Q code over
  GF(256) with the polynomial 0x11D (Sections 4.1, 4.2).
"""

from . import ring, zp_raid, rs_gf256  # noqa: F401
