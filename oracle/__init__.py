"""Plain FP64 CPU oracle for the lattice Boltzmann particle-coupling hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything under ``oracle/``.  The
product path (the HIP library and its Python binding) never imports, links or
calls this package, and this package never imports the product package.

What it computes follows Rettinger & Ruede, "A comparative study of
fluid-particle coupling methods for fully resolved lattice Boltzmann
simulations" (arXiv:1702.04910):

* ``lattice``  -- D3Q19 velocities and weights (Sec. 2.1).
* ``fluid``    -- moments, incompressible equilibrium (Eq. LBM_EQ), BGK
                  (Eq. LBM_SRT), TRT (Eq. MEM_TRT), forcing (Eq. Forcing),
                  macroscopic velocity (Eq. MacVel), streaming (Eq. LBM_Stream).
* ``geometry`` -- sphere mapping, wall distance delta_q, supersampled solid
                  fraction (Sec. 2.3.2), flat and recursive.
* ``psm``      -- partially saturated cells collision (Eqs. PSM, PSM_B1/B2,
                  PSM_M1..M3, LBM_Collide_PSM, MacVel_PSM) and force/torque
                  (Eqs. PSM_TotForce, PSM_TotTorque).
* ``mem``      -- momentum exchange: bounce-back (Eq. MEM_BB), CLI
                  (Eq. MEM_CLI), link force (Eq. MEM_Force), totals
                  (Eqs. MEM_TotForce/TotTorque), refill (Eq. MEM_Reconstruction).
* ``rigid``    -- explicit Euler rigid-body update (Sec. 4.1).
* ``sim``      -- the two drivers, Alg. 1 (MEM) and Alg. 2 (PSM).
* ``mlp``      -- FP64 reference forward/backward of the solid-fraction MLP.

Storage convention: every PDF is held as the deviation g_q = f_q - w_q from the
lattice weight (f = w + g exactly); each function states how the paper's
equation reads in that variable.  Arrays are indexed ``g[q, z, y, x]``.

Parity status: every function is pinned by a ``-m "not gpu"`` test against a
closed form, an invariant, a brute-force count or a value printed in the paper,
except the items marked "parity unpinned" in their docstrings (refill tie
rules, MLP design choices).
"""
