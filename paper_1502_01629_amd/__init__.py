"""MI355X-native semi-Lagrangian solver for second-order HJB equations (arXiv 1502.01629)."""
