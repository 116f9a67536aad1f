"""CPU oracle for exact Strassen-Winograd products over Z/pZ.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import, call, link or execute anything in this package.
It shares no code with the GPU library, and the product path never reaches it.

* ``ref``       -- O1, the plain value (alpha*A*B + beta*C) mod p, in C.
* ``schedules`` -- O2, Winograd's algorithm replayed under each memory
                   schedule of the paper (Tables 1-9, Algorithm 2), with
                   operation counts and a temporary-memory arena.
* ``limbs``     -- O4, balanced base-256 digits of centred residues and the
                   product recombined from digit products.
"""
