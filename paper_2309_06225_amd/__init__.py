"""MI355X-native 4dST/CCZ4 right-hand side and RK4 hot path (libgrf)."""
