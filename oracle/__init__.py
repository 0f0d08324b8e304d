"""FP64 CPU oracle for the exact O(mM) belief-propagation update.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link this package; only the tests,
the smoke check and the benchmark's CPU-baseline leg use it.  It shares no
code with the GPU path: the only common module is ``synth_mrf``, which draws
inputs and holds none of the method's arithmetic.

Modules
-------
grid_bp   pairwise BP on a 4-connected grid; dense, split and sparse message
          forms for sum- and max-product; synchronous and checkerboard
          schedules; beliefs and MAP labels.
graph_bp  plain dense BP on an arbitrary undirected graph (edge list).
brute     exhaustive marginals, max-marginals and MAP of tiny MRFs.
grad_ref  hand-written adjoint of unrolled synchronous sum-product BP on the
          grid, FP64.
torch_bp  an independent differentiable forward (plain PyTorch CPU ops, FP64)
          used only to cross-check grad_ref through autograd.
"""
