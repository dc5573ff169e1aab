"""FP64 CPU oracle of the coupled LB crystal-growth step. TEST INFRASTRUCTURE ONLY."""
