"""MI355X-native aSP-AMG solve phase (PCG + adaptive AMG V-cycle) for 3x3-block elasticity systems."""
