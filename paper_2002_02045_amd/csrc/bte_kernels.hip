// BTE kernels
namespace ephx {}
