"""Plain FP64 CPU oracle for the rational-program fit, evaluation and argmin.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the benchmark's
CPU-baseline leg may import this package.  The product path (the HIP library and its Python
binding) never imports, calls or links anything here, and this package imports nothing from the
product path: the two share only the seeded input generators.

Modules:
  fit   - linearised rational least squares by column-pivoted Householder QR
          (section "Building a Driver Program: Rational function estimation")
  cost  - occupancy flowchart (Example "Hardware occupancy", eq. occupancy), the MWP-CWP-style
          cycle estimate, brute-force argmin (steps 4 and 5 of section "An Algorithm to Build
          and Deploy a Performance-Predicting Rational Program")
  mlp   - FP64 forward / backward / Adam of the surrogate network
"""
