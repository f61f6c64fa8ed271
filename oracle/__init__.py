"""CPU oracle for the compressed-graph product and PageRank.

TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's
CPU-baseline leg import this package.  It shares no code with the HIP
library; both sides read the same seeded inputs (``bvinputs``).

Modules:
  bvdecode  - independent decoder of the project's BV-style bitstream
  product   - y = A x (plain definition) and the paper's sequential reuse
              algorithm on the difference form (A', r)
  pagerank  - power method, Eq. (1) of the paper, and a dense solve
  biclique  - the biclique format of Section "Final Remarks": the lists it
              stands for, and the paper's two-step product
"""
from . import biclique, bvdecode, pagerank, product  # noqa: F401
