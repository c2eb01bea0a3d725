"""CPU FP64 oracle for the adaptive point-charge Laplace FMM.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use
it.  It shares no code, tables or helpers with the HIP library in
``paper_2511_15269_amd/``; the only common input is the seeded generator
module ``workloads.py``, which holds no arithmetic of the method.

Modules (each function cites the passage of the paper it follows):

* ``direct``       -- the O(N^2) direct sum (eqs. 1-3) and its gradient
* ``basis``        -- regular/singular solid harmonics: closed forms from their
                      definitions (App. A) and the App. A recursions
* ``expansions``   -- multipole and local expansions (eqs. 9-12 and the real
                      form of Sec. II.C)
* ``translations`` -- the direct O(p^4) multipole-to-local operator
* ``tree``         -- the balanced median-split 2^s tree (Sec. II.A)
* ``lists``        -- admissibility (eq. 4) and the cross-level level-marching
                      interaction lists (Sec. II.B)
* ``fmm``          -- the FMM assembled from the above
* ``gradient``     -- derivatives of E = 1/2 sum q_i u_i

Readings taken where the paper is silent or garbled are stated at the point
of use, each marked "Reading:".
"""
