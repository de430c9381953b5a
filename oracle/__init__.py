"""Plain CPU FP64 HOTRG oracle -- TEST INFRASTRUCTURE ONLY.

This package is the correctness reference that the HIP path is checked
against.  It is deliberately slow and obvious: NumPy in float64, LAPACK eigh,
no blocking or fusion beyond the contraction order spelled out in each
function.  It shares no code, header, table or helper with the product package
(`paper_1906_06060_amd`), and the product never imports it.  Only `tests/`,
`__graft_entry__.smoke()` and the `cpu_baseline` leg of `bench.py` may import
or execute anything in here.

Modules
-------
hotrg   : the HOTRG method (Akiyama, Kuramashi, Yamashita, Yoshimura,
          "Phase transition of four-dimensional Ising model with HOTRG",
          Sec. 2), d-generic (d = 1..4), with the impurity method and the
          X^(n) indicator (Sec. 3, Eqs. (3.2)-(3.3)).
exact   : closed forms and brute force used to pin the oracle (transfer
          matrix in d = 1, Onsager in d = 2, enumeration of tiny tori,
          high-temperature series).
sample  : single entries / row blocks of one coarse-graining step computed
          straight from the definition, for parity at sizes where a full
          oracle step is too slow.
tangent : forward-mode derivative of ln Z / N through the whole flow
          (including the eigenvector derivative), independent of any
          reverse-mode code.
tc      : T_c(Dcut) by bisection on the settled X^(n) of pure-tensor flows
          (Sec. 3).
jump    : energy and magnetisation jumps at T_c from two-sided straight
          lines, m taken to zero field from two small fields (Sec. 3).

Pins: every function is pinned by tests in `tests/test_oracle_*.py` against
values fixed by the paper or by mathematics.  Functions without such a pin say
"parity unpinned" in their docstring.
"""
