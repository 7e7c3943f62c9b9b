"""CPU FP64 oracle for the implicit-Euler finite-volume reaction-diffusion solve.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it; the library and its
Python binding never do, and it shares no code, headers, tables or helpers with
them.  Inputs come from the seeded generators in ``synth`` (data only).

Modules (each function cites the paper passage it follows):

* ``bbox``   - bounding box of the tumour cells plus a margin (Sec. 2.3);
* ``fv``     - cell-centred finite-volume assembly of one implicit-Euler step of
               dc/dt = div(D grad c) - k c + s on the box (Sec. 2.2, eqs. 1-4;
               Sec. 2.4);
* ``krylov`` - dense LU, Jacobi-preconditioned CG and restarted GMRES with
               modified Gram-Schmidt (Sec. 2.4, GMRES of Saad and Schultz);
* ``step``   - the whole step: box, assembly, solve, write-back onto the mask
               (Sec. 2.3-2.4);
* ``unet``   - FP64 forward/backward of the warm-start U-Net (not in the paper;
               its architecture is part of this project's specification).

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
invariants, hand-derived fixtures or library routines; see the module headers.
"""
