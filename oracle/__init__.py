"""CPU oracle for the full multigrid method for semilinear elliptic equations.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import this package:
only the test-suite, the smoke check and the benchmark's CPU-baseline leg use it.
It shares no code with the HIP library (the only common module is the seeded
input generator `paper_1611_05677_amd.workloads`, which holds no solver
arithmetic).

Everything here is plain, slow and written to be checked by eye against the
paper: element-by-element P1 assembly into CSR matrices (Section 2, eq.
"FEM_form"), a fine-space Newton solve (O1, `o1.py`), and a replica of the
one-correction-step and full-multigrid algorithms (O2, `o2.py`; Section 3,
Algorithms 3.1 and 3.2), in float64.
"""
