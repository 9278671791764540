"""Plain FP64 CPU oracle for the inverse matrix p-th root iteration.

TEST INFRASTRUCTURE. Only the test suite, the package smoke check and the
bench's CPU-baseline leg may import, call or execute anything in this package.
The product (the HIP library and its Python binding) never uses it, and it
shares no code with the product: no kernels, helpers, tables or constants. The
only module both sides use is ``workloads`` (seeded input generators, which
hold none of the method's arithmetic).

Everything here is written for a reader to check against the paper by eye:
NumPy float64, one library primitive per step (matmul, eigh), no blocking, no
fusion, no reordering beyond what the cited passage states.

Parity pins (tests marked "not gpu" check each of these):
  * ``eig_root``       - against scipy.linalg.fractional_matrix_power, a
                         hand-worked 2x2 closed form, diagonal closed form.
  * ``solve``          - against eig_root, numpy.linalg.inv (p = 1), the
                         scalar recursion on diagonal and scaled-identity A
                         (bit for bit), spectral iteration counts, invariants;
                         its floor rule's zone against the closed forms of
                         one step's contraction (p = 1, 2).
  * ``spectral_count`` - against the dense iteration's count.
  * rounding emulator  - against torch dtype casts (bf16, fp16, fp8 e4m3).
  * MLP forward/back   - backward against central finite differences; GELU
                         against its closed form values.
  * features           - against hand-computed values on small matrices.
  * guard              - against dense sampling and the closed forms of the
                         paper's eq. (3) start.
  * int8-slice product - against exact integer and rational arithmetic
                         (brute force on tiny inputs) and its error bound.
  * approximate storage - against the scalar recursion on diagonal A, the
                         stored-bit floors and the behaviour Section IV-C reports.
  * all arithmetic     - the rounded product against brute-force scalar loops
                         with a separately written rounding rule, the rounded
                         scalar recursion on diagonal A (bit for bit), 52 bits
                         against the float64 iteration, floors above the
                         storage-only regime's (Section IV-C).
  * scaled steps       - the factor against its closed forms (p = 1, 2) and
                         brute force over whole spectra; the dense count
                         against the per-eigenvalue count.
  * Loewdin transform  - against scipy's generalised eigenvalues and closed
                         forms.
Parity unpinned: none of the functions above lacks a pin. The accuracy the
low-precision bulk phase reaches end to end has no value in the paper to
compare with (its figures are not available); it is checked against this
oracle's emulator only.
"""
