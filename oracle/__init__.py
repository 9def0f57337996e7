"""Plain FP64 CPU oracle for the alpha-Moebius domain-wall propagator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (no kernels, layouts, tables or helpers); the two meet only through the
seeded input arrays of ``paper_1501_04950_amd.synth``.

The oracle is written to be checked by eye against the paper (H. Neff, "A
better conditioned Domain Wall Operator"):

* ``gamma``    -- Dirac matrices and chiral projectors P+- (eq. (coeff)).
* ``wilson``   -- the Wilson operator D_w of eq.(wilson), written out literally
                  on full-lattice complex128 arrays, and its adjoint stencil.
* ``mobius``   -- D_alpha(m) as the literal block matrix of eq.(mobius1), the
                  conventional Moebius operator it reduces to at alpha = 1, and
                  the matrices P (eq.(eqP)) and A (Sec. 2).
* ``redblack`` -- the red-black form D_bb = 1 - I_bb^-1 D_br I_rr^-1 D_rb of
                  eq.(redblack), its adjoint, CG on the normal equations, and
                  the propagator y_1 of eq.(tosolve)/(tosolve1).
* ``adjoint``  -- gradients of L = Re <eta', y_1> with respect to the links,
                  the source, alpha, b_i and c_i by the adjoint-state method,
                  term by term from the block matrix of eq.(mobius1).
* ``overlap``  -- dense and closed-form tools used only as pins: the dense
                  transfer-matrix overlap operator of Appendix A and the free
                  field momentum-space operator.

Everything is complex128 and follows the paper's order of operations; numpy
routines (einsum, roll, inv, solve) serve as library primitives only.
"""
