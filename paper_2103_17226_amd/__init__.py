"""Batched arithmetic-circuit evaluation for noisy variational quantum
circuits on MI355X (gfx950).

Huang, Holtzen, Millstein, Van den Broeck, Martonosi, "Logical Abstractions
for Noisy Variational Quantum Algorithm Simulation", ASPLOS 2021: a noisy
circuit is compiled (circuit -> Bayesian network -> CNF -> arithmetic
circuit, Sec. 3.1-3.2) once on the host, and the arithmetic circuit is then
evaluated many times on the GPU for amplitudes (upward pass, Sec. 3.3.1),
derivatives and Gibbs samples (downward pass, Sec. 3.3.2).

Modules:
  compiler  -- host preprocessing: circuit -> BN -> CNF -> level-ordered AC
  blob      -- serialisation of the AC for the C ABI
  _lib      -- ctypes view of include/qkc.h
  api       -- ACGraph (eval / grad / sample) and the autograd wrapper
  serve     -- continuous-batching request loop over resident graphs
  build     -- hipcc build of libqkc.so
"""
