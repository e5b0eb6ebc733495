"""Generator of the pointwise device code (forward right-hand side and its VJP)."""
