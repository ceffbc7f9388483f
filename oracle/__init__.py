"""FP64 CPU oracle for the scatter-accumulate reverse-mode path.

TEST INFRASTRUCTURE ONLY. Nothing in the product package may import, link or
call this package; only the test-suite, the smoke entry and the CPU-baseline leg
of the benchmark do. It shares no code with the HIP path: the two meet only in
the seeded input generators (``workloads``), which hold none of the method's
arithmetic.

Everything here is plain, slow and in float64. Library primitives (a matrix
product, a sum) serve as single steps; there is no blocking, fusion or
reordering beyond what the definitions state.

Paper: "Getting to the Point. Index Sets and Parallelism-Preserving Autodiff for
Pointful Array Programming" (arXiv 2104.05372).

Modules
  gmm      GMM log-likelihood objective and its gradient (transpose of the
           linearized map, Sec. 5.1-5.2).
  scatter  indexed read (gather) and its transpose, the `+=` accumulation into a
           sliced reference (Sec. 2.3.2-2.3.3, Sec. 5.3.3; rule
           LetIndexingTranspose, Fig. "transposition rules"); histogram
           (Sec. 6.1.2).
  stencil  in-place (State) diffusion loop and its transposed loop (Sec. 2.3.1,
           Sec. 5.3.2; rules ForTranspose / GetTranspose / PutTranspose).
"""
from . import gmm, scatter, stencil  # noqa: F401
