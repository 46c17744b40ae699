"""CPU oracle for state-vector gate application.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product library
(``paper_1805_04708_amd``) never imports it, and the two share no code: the
oracle has its own gate table (``oracle.gates``), its own C kernels
(``oracle/jq_oracle.c``) and its own dense brute force (``oracle.dense``).

Functions without an independent pin are marked "parity unpinned" in their
docstrings.
"""
