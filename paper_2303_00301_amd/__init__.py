"""MI355X-native auxiliary Kalman MCMC (parallel-in-time filter and sampler)."""
