"""MI355X-native phylogenetic log-likelihood and branch-length gradient."""
