"""CPU oracle for the dynamic-circuit state-vector path (complex128, NumPy).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything from this package. It
shares no code with the product library (``paper_2604_11599_amd``) and imports
nothing from it; the only module both sides use is the seeded input generator
package ``workloads``, which holds no simulation arithmetic.

Modules:
  philox  Philox4x64-10 from its published definition; per-shot event streams.
  gates   gate matrices and their angle derivatives.
  qasm    an OpenQASM 3 subset parser producing a tuple AST.
  sim     the tree-walking state-vector interpreter, expval, gradients.
  brute   dense 2^n x 2^n operators and projectors (n <= 8) for cross-checks.
"""
