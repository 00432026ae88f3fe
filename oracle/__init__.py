"""Plain FP64 CPU oracle for the constrained DTT/FFT elasticity solver.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code with
the GPU library: everything here is written from the paper (Gelebart &
Amouzou-Adoun, "Constrained minimization problems and FFT-based solvers"),
with NumPy/SciPy primitives (matmul, DCT/DST, dense/sparse solves) as steps.

Modules
  dtt      discrete trigonometric transforms per boundary type (Tables 1-3, eq 7)
  plan     boundary table -> symmetries, transform types, A-DOFs, boundary weights
  tetra2   TETRA2 scheme: element gradients, stress, nodal divergence, assembly
  green    reference-medium symbol from the assembled stencil, Green solve (eq 3-4)
  solver   Algorithm 1 (equality constraints) with Anderson acceleration
  contact  Algorithm 2 (small-strain unilateral contact, active set)
  kkt      direct solves of the constrained minimisation (eq 18-23, 31-33)
  nn       FP64 reference of the warm-start network with a hand-written backward

Parity status of each function is stated in its docstring; functions pinned
only against their own reading of an underspecified passage say
"parity unpinned".
"""
