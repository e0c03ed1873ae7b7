"""MI355X-native runtime construction of spiking-network connectivity."""
