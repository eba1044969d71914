"""MI355X-native differentiable underwater Gaussian rasterizer."""
