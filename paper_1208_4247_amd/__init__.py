"""MI355X-native geometric multigrid for the finite-difference Poisson problem."""
