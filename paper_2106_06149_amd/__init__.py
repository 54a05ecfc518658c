"""MI355X-native MBE(3)-OSV-MP2 per-cluster hot path (arXiv 2106.06149).

synth     seeded synthetic inputs (shared by the library's tests and the oracle)
api       OSVContext: build / solve / energy / densities through libosvmbe.so
autograd  OSVEnergy, a torch.autograd.Function with the hand-written adjoint
"""
