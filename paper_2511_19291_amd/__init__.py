"""MI355X-native state-vector simulator: the single-GPU hot path of the
method of "TorchQuantumDistributed" (gates on a dense complex state, Pauli
expectation values, adjoint gradients, batched circuits).

Submodules:
  circuits  -- seeded synthetic circuits and observables (plain data)
  sv        -- ctypes binding of the HIP library libsv.so (C ABI in include/sv.h)
  autograd  -- torch.autograd.Function over the adjoint backward

Importing this package does not load the GPU library; ``sv`` does, and
raises if it is missing.
"""

__all__ = ["circuits"]
