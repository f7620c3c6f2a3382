"""CPU oracle for the cumulant lattice Boltzmann hot path and the FNO surrogate.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute anything
in this package.  The product library (``paper_2606_16765_amd``) never does:
it shares no code, header, table or helper with this package.

Modules:
  lbm    ctypes wrapper of ``lbm_oracle.c`` (FP64, two-lattice pull scheme)
  brute  numpy brute-force variant (27x27 moment matrix, generic set-partition
         cumulants) used to pin ``lbm`` on small boxes
  fno    numpy FP64 Fourier Neural Operator: forward, hand-written adjoints,
         masked MSE and Adam
"""
