"""CPU oracle for the Generalized Fermat prime field FFT and polynomial product.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding, the request loop) may import, call, link or execute anything
in this package.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.

Everything here is plain and slow on purpose: Python integers, exact
arithmetic modulo p, definitions written out (the DFT as a sum, the product
of polynomials as a double loop), and the paper's algorithms taken step by
step in the paper's order and notation where the paper gives an algorithm
rather than a definition.  It shares no code with the HIP path.

Modules
-------
primality   Baillie-PSW probable-prime test (Miller-Rabin base 2 + strong
            Lucas with Selfridge parameters).
field       The field Z/pZ for p = r^k + 1 (section 2 of the paper): radix-r
            encoding, plain modular arithmetic, the paper's element
            algorithms (Alg. 2 addition, multiplication by a power of r,
            Alg. 3 multiplication) and the primitive root of Alg. 1.
transform   DFT / inverse DFT by definition, a textbook radix-2 NTT for
            larger sizes, the paper's Algorithm DFT_general (section 4.3),
            the tensor-algebra operators of section 4.1, Horner evaluation
            and the schoolbook polynomial product.

Parity status: every function here is pinned by tests under ``tests/``
(test_oracle_*.py) against facts fixed by the paper or by mathematics;
none is "parity unpinned".
"""
