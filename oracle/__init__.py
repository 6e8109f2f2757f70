"""CPU oracle for the exact multiprecision Hankel / Toeplitz / circulant matvec.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
executes this package; only the test-suite, the smoke check and the
benchmark's CPU-baseline leg do.  It shares no code with the HIP path.

Everything here is plain, slow and exact: Python integers (and
`fractions.Fraction` in the pins), no floating point in the arithmetic.

Modules
  fixedpoint     word encoding of P-bit fixed-point numbers, round-half-even
  hankel         schoolbook products (Preliminaries, eqs. (1)-(3) and the
                 schoolbook sum) -- the definition the fast paths must equal
  alg1           the recursive half-size scheme of Section 4 (Algorithm 1)
                 in exact integers, and its multiplication count
  decomposition  the exact integer analogue of the Section 3 decomposition
                 (numbers as sums of limbs, one bivariate correlation)
  kronecker      a fast exact cross-check: the whole matvec as one GMP
                 big-integer product (Kronecker substitution)
"""
