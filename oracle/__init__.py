"""CPU oracle for the optimal cycle mean.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark, never by the library.  It shares no code with the
HIP path; both sides only consume the same generated input arrays.

* ``brute``    simple-cycle enumeration in exact rationals (tiny graphs);
* ``native``   ctypes wrapper of ``ocm_oracle.c``: Karp, sequential policy
               iteration (Alg. 2), exact tie test, optimality certificate;
* ``closed``   closed forms (ring, self-loops, product of local automata).
"""
