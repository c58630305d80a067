"""Kernel-variant tuner: the variant space of the Euler-step kernels, a benchmark harness,
an append-only individual database, and four search strategies (exhaustive, random,
the paper's parallel asynchronous genetic simulated annealing, and an MLP cost model
trained on the GPU that proposes variants before they are benchmarked)."""
