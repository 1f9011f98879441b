"""MI355X-native differentiable synchrotron sightline march (arXiv:2410.01136)."""
