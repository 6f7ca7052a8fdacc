"""MI355X-native Vecchia Gaussian-process log-likelihood, gradient and Fisher information."""
